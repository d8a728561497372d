// Run detection and the leaf partition (Sec. 2 run convention; Alg. PowerSort
// with the minimum-run extension of App. B.4).
//
// Sequentially, the leaves are the orbit of position 0 under
//     J(s) = min(segEnd(s), max(runEnd(s), s + w)),
// where runEnd(s) is the end of the natural run that starts at s (weakly
// increasing, or strictly decreasing) on the ORIGINAL data: a merge only
// touches positions left of the next run start and a min-run extension only
// positions inside its own leaf, so the partition never depends on data the
// algorithm has already moved.
//
// In parallel: tile t = [T0, T1) of kPartTile positions is entered by the
// chain at one of w+1 candidate points: T0 + c for c < w, or the end X0 of the
// natural run that crosses T0 (the only way the chain can jump further).  For
// each candidate the tile records the candidate through which the chain
// leaves (an "exit code" into the next tile) and how many leaf starts it
// visits.  These small tables compose associatively; a hierarchical scan over
// them yields each tile's true entry, and a second pass over the tile emits
// the leaf starts.
//
// Inside a tile the chain is followed in one of four ways: a tile inside
// one long run jumps straight past its window; a tile with few run changes
// and segment starts (at most kWalkMax) walks each chain point by point,
// finding J from short sorted lists of those positions; a tile whose natural
// runs are all shorter than w steps by w (an arithmetic progression); any
// other tile resolves J for every position and follows it by pointer
// jumping.
#include "common.hpp"
#include "block.hpp"
#include "internal.hpp"

namespace ps {

constexpr int kPairItems = 17;                     // pairs per thread in the window scan
constexpr int kPairCap = kThreads * kPairItems;    // 4352 >= kPartTile + kMaxMinRun + 2
static_assert(kPartTile % kSampleSpacing == 0 && kPartTile / kSampleSpacing <= kThreads,
              "a partition tile starts at a sampled position, and one thread stores each of its samples");
constexpr uint32_t kFar = 0xFFFFFFFEu;             // a position beyond the tile's window (!= kInf)
constexpr uint16_t kExitBit = 0x8000u;
// kWalkMax (internal.hpp): a chain never takes more steps in a tile than the
// tile holds run changes and breaks, plus one: every step lands on or passes
// one of them.

enum : uint8_t { kAsc = 0, kDesc = 1, kBreak = 2, kUnknown = 3 };
// How tile_successors left the tile.
enum : int { kTileTable = 0, kTileUniform = 1, kTileWalk = 2, kTileDense = 3 };

// First entry above v of the ascending list a[0..n), or kInf.
__device__ __forceinline__ uint32_t first_above(const uint16_t* a, uint32_t n, uint32_t v) {
    uint32_t lo = 0, hi = n;
    while (lo < hi) {
        const uint32_t m = (lo + hi) >> 1;
        if (a[m] <= v) lo = m + 1; else hi = m;
    }
    return lo < n ? (uint32_t)a[lo] : kInf;
}

template <int KT>
struct PartShared {
    using U = typename Key<KT>::ukey;
    union {
        struct {
            uint16_t nx[kPartTile];           // successor (or exit) per tile position
            uint16_t ct[kPartTile];           // leaf starts up to the exit
        } pj;
        struct {
            uint16_t nx[kPartTile];
            uint8_t mk[kPartTile];            // chain-point marks
        } em;
    } u;
    U edge[kWaves][kPairItems + 1];           // each wave's lane-0 keys (the previous wave's right neighbours)
    uint8_t pt[kPairCap];                     // pair type of pair (T0-1+k, T0+k)
    uint16_t chg[kWalkMax];                   // walk: pairs k > 0 whose type differs from pair k-1
    uint16_t brk[kWalkMax];                   // walk: pairs k of type kBreak
    uint8_t ctype[kWalkMax];                  // walk (emit): type of pair chg[i]
    uint32_t nchg, nbrk;
    uint32_t dirs;                            // OR of the directions seen: 1 ascending, 2 descending
    uint32_t sh[2 * kWaves];
    uint32_t gfirst;
    uint32_t x0;                              // end of the run crossing T0 (kFar / kInf)
    uint32_t smp[kPartTile / kSampleSpacing]; // order keys of the tile's sampled positions
};

// Classifies pairs of tile [T0, T1) and its window and sets sm.x0, the end of
// the natural run crossing T0 (kInf if none, kFar if beyond the window).
// Returns
//  * kTileUniform when the whole tile lies inside one natural run that
//    extends past the window: every J(s) is the run's end, beyond the
//    window (exit code w);
//  * kTileWalk when the window holds at most kWalkMax run changes and breaks
//    together: they are listed in sm.chg / sm.brk, and walk_next gives J;
//  * kTileDense when no break lies in the window and every natural run
//    starting in the tile is shorter than w: then J(s) = s + w for every s;
//  * kTileTable otherwise, with the encoded successor of every position s in
//    sm.u.pj.nx (aliased by sm.u.em.nx): a tile-local index if J(s) < T1,
//    else kExitBit | exit code.
template <int KT>
__device__ __forceinline__ int tile_successors(const typename Key<KT>::raw* __restrict__ keys, uint32_t N,
                                const uint64_t* __restrict__ offsets, uint32_t nseg,
                                const uint32_t* __restrict__ tile_seg, uint32_t w,
                                uint32_t T0, uint32_t T1, PartShared<KT>& sm,
                                uint32_t* __restrict__ samp = nullptr) {
    using K = Key<KT>;
    using U = typename K::ukey;
    const int tid = threadIdx.x;
    // Window: positions [T0-1, WE) as indices [0, NPW); pair k = (T0-1+k, T0+k).
    const uint32_t WE = (uint32_t)min<uint64_t>((uint64_t)N, (uint64_t)T1 + w + 1);
    const uint32_t NPW = WE - T0 + 1;  // number of positions in the window = pairs

    {
        // All of this thread's window loads are issued before the first use.
        // Lane L holds window index tid + i * kThreads; its right neighbour
        // is lane L+1's, or, for a wave's last lane, the next wave's lane 0
        // (passed through LDS).  The pair types are computed in registers:
        // the keys themselves never go to LDS.
        const int lane = tid & 63, wv = tid >> 6;
        typename K::raw kv[kPairItems];
#pragma unroll
        for (int i = 0; i < kPairItems; ++i) {
            const uint32_t k = tid + i * kThreads;
            if (k < NPW && !(k == 0 && T0 == 0)) kv[i] = keys[T0 - 1 + k];
        }
        if (sizeof(U) == 4 && samp) {
            // the tile's sampled positions (T0 is a multiple of the spacing),
            // kept in LDS: the caller stores them after its last barrier
#pragma unroll
            for (int i = 0; i < kPairItems; ++i) {
                const uint32_t k = tid + i * kThreads;
                if (k >= 1 && T0 - 1 + k < T1 && ((k - 1) & (kSampleSpacing - 1)) == 0)
                    sm.smp[(k - 1) / kSampleSpacing] = (uint32_t)K::ord(kv[i]);
            }
        }
        if (lane == 0) {
#pragma unroll
            for (int i = 0; i < kPairItems; ++i) sm.edge[wv][i] = K::ord(kv[i]);
        }
        if (tid == 0) {
            if (nseg > 1) sm.gfirst = tile_seg[T0 / kPartTile];  // first offset >= T0
            sm.dirs = 0;
        }
        __syncthreads();
        // pair types of this thread's pairs, 2 bits each, kept in registers
        // until the tile is known not to lie inside one run
        uint64_t types = 0;
        uint32_t dirs = 0;
#pragma unroll
        for (int i = 0; i < kPairItems; ++i) {
            const uint32_t k = tid + i * kThreads;
            const U u = K::ord(kv[i]);
            U v = __shfl_down(u, 1);
            if (lane == 63) v = (wv + 1 < kWaves) ? sm.edge[wv + 1][i] : sm.edge[0][i + 1];
            uint32_t t;
            if (k == 0 && T0 == 0) {
                t = kBreak;                                  // nothing left of position 0
            } else if (k + 1 < NPW) {
                t = (v < u) ? kDesc : kAsc;
                if (k >= 1) dirs |= (t == kDesc) ? 2u : 1u;
            } else {
                t = (WE == N) ? kBreak : kUnknown;           // pair (WE-1, WE)
            }
            types |= (uint64_t)t << (2 * i);
        }
        // one LDS word gathers the directions: a wave OR, then one atomic per wave
        const uint32_t wdirs = (__ballot(dirs & 1u) ? 1u : 0u) | (__ballot(dirs & 2u) ? 2u : 0u);
        if (lane == 0 && wdirs) atomicOr(&sm.dirs, wdirs);
        __syncthreads();
        // Inside one long run?  Every pair 1..NPW-2 has one direction, the
        // window ends before N, and no segment starts inside it.
        const uint32_t all = sm.dirs;
        const bool seg_inside = nseg > 1 && sm.gfirst <= nseg && offsets[sm.gfirst] <= (uint64_t)WE;
        if ((all == 1u || all == 2u) && WE < N && !seg_inside) {
            if (tid == 0) {
                // the run through pair (T0-1, T0) either continues (same
                // direction), or does not exist (a break), or ends at T0
                const uint8_t t0 = (uint8_t)(types & 3u), t1 = (all == 2u) ? (uint8_t)kDesc : (uint8_t)kAsc;
                sm.pt[0] = t0;
                sm.x0 = (t0 == t1) ? kFar : (t0 == kBreak ? kInf : T0 + 1);
            }
            __syncthreads();
            return kTileUniform;
        }
#pragma unroll
        for (int i = 0; i < kPairItems; ++i) {
            const uint32_t k = tid + i * kThreads;
            if (k < NPW) sm.pt[k] = (uint8_t)((types >> (2 * i)) & 3u);
        }
        __syncthreads();
    }
    // A segment start o in (T0-1, WE] breaks pair o-1: runs never cross it.
    // (With one segment the only starts are 0 and N, handled above.)
    for (uint32_t g = sm.gfirst + tid; nseg > 1 && g <= nseg; g += kThreads) {
        const uint64_t o = offsets[g];
        if (o > (uint64_t)WE) break;
        if (o >= 1 && o >= (uint64_t)T0) sm.pt[(uint32_t)(o - T0)] = kBreak;
    }
    __syncthreads();

    // Per thread: pairs k = tid*kPairItems + i.
    uint8_t tp[kPairItems];
    uint32_t cpos_min = kInf, bpos_min = kInf;
    uint32_t counts = 0;  // changes << 16 | breaks
#pragma unroll
    for (int i = 0; i < kPairItems; ++i) {
        const uint32_t k = tid * kPairItems + i;
        tp[i] = (k < NPW) ? sm.pt[k] : kUnknown;
        const bool chg = (k < NPW) && k > 0 && tp[i] != sm.pt[k - 1];
        if (chg) cpos_min = min(cpos_min, k);
        if (k < NPW && tp[i] == kBreak) bpos_min = min(bpos_min, k);
        counts += (chg ? (1u << 16) : 0u) + ((k < NPW && tp[i] == kBreak) ? 1u : 0u);
    }
    uint32_t nbreaks;
    {
        uint32_t tot;
        const uint32_t ex = block_excl_sum(counts, sm.sh, &tot);
        nbreaks = tot & 0xFFFFu;
        if ((tot >> 16) + (tot & 0xFFFFu) <= kWalkMax) {
            // Few changes and breaks: list them in position order.
            uint32_t oc = ex >> 16, ob = ex & 0xFFFFu;
#pragma unroll
            for (int i = 0; i < kPairItems; ++i) {
                const uint32_t k = tid * kPairItems + i;
                if (k < NPW && k > 0 && tp[i] != sm.pt[k - 1]) sm.chg[oc++] = (uint16_t)k;
                if (k < NPW && tp[i] == kBreak) sm.brk[ob++] = (uint16_t)k;
            }
            if (tid == 0) {
                sm.nchg = tot >> 16;
                sm.nbrk = tot & 0xFFFFu;
            }
            __syncthreads();
            if (tid == 0) {
                // the run through pair 0 crosses T0 unless that pair is a break
                const uint8_t t0 = sm.pt[0];
                if (t0 == kBreak) sm.x0 = kInf;
                else if (t0 == kUnknown) sm.x0 = kFar;
                else {
                    const uint32_t kc = first_above(sm.chg, sm.nchg, 0u);
                    sm.x0 = (kc == kInf || sm.pt[kc] == kUnknown) ? kFar : T0 + kc;
                }
            }
            __syncthreads();
            return kTileWalk;
        }
    }
    const uint32_t cex = block_excl_suffix_min(cpos_min, sm.sh);
    const uint32_t bex = block_excl_suffix_min(bpos_min, sm.sh + kWaves);
    uint32_t runc = cex, runb = bex;
    // One right-to-left pass gives, for every pair k of this thread, the next
    // type change after k (runc) and the next break at or after k (runb), and
    // with them the successor J of position T0-1+k, written to nx.  It also
    // decides the dense case: every natural run starting in the tile shorter
    // than w and no break in the window, so J(s) = s + w throughout (then nx
    // is not used).
    bool any_long = false;
    const uint32_t len = T1 - T0;
#pragma unroll
    for (int i = kPairItems - 1; i >= 0; --i) {
        const uint32_t k = tid * kPairItems + i;
        const uint32_t kc = runc;  // first change after k
        if (k < NPW && k > 0 && tp[i] != sm.pt[k - 1]) runc = k;
        if (k < NPW && tp[i] == kBreak) runb = k;
        const uint32_t kb = runb;  // first break at or after k
        if (k >= NPW) continue;
        // the run from position T0-1+k (k in [1, len]) ends at T0 + kc
        if (k >= 1 && k <= len && (kc == kInf || sm.pt[kc] == kUnknown || kc - k + 1 >= w)) any_long = true;
        // End of the run containing pair k, as a position (kFar if unknown).
        uint32_t ne;
        if (tp[i] == kBreak) ne = T0 + k;  // the run starting at T0-1+k is that single element
        else if (tp[i] == kUnknown) ne = kFar;
        else ne = (kc == kInf || sm.pt[kc] == kUnknown) ? kFar : (T0 + kc);
        if (k == 0) {
            // Run crossing T0: only a real (non-break) pair (T0-1, T0) crosses.
            sm.x0 = (tp[i] == kBreak) ? kInf : ne;
            continue;
        }
        const uint32_t s = T0 - 1 + k;
        if (s >= T1) continue;
        const uint32_t seg_end = (kb == kInf) ? kFar : (T0 + kb);
        uint32_t J;
        if (ne == kFar) J = kFar;
        else if (ne - s >= w) J = ne;
        else J = min(seg_end, s + w);
        uint16_t enc;
        if (J < T1) enc = (uint16_t)(J - T0);
        else enc = kExitBit | (uint16_t)((J != kFar && J - T1 < w) ? (J - T1) : w);
        sm.u.pj.nx[s - T0] = enc;
    }
    // the block-wide OR is also the barrier after every nx and x0 write
    const bool dense = __syncthreads_or(any_long) == 0 && nbreaks == 0;
    return dense ? kTileDense : kTileTable;
}

// J(s) for a position s in [T0, T1) of a tile in walk mode: the same rule as
// the per-position table, with the next change and break from the lists.
template <int KT>
__device__ __forceinline__ uint32_t walk_next(const PartShared<KT>& sm, uint32_t T0, uint32_t s, uint32_t w) {
    const uint32_t k = s - T0 + 1;  // pair (s, s+1)
    const uint8_t t = sm.pt[k];
    uint32_t ne;
    if (t == kBreak) {
        ne = s + 1;
    } else if (t == kUnknown) {
        ne = kFar;
    } else {
        const uint32_t kc = first_above(sm.chg, sm.nchg, k);
        ne = (kc == kInf || sm.pt[kc] == kUnknown) ? kFar : T0 + kc;
    }
    if (ne == kFar) return kFar;
    if (ne - s >= w) return ne;
    const uint32_t kb = first_above(sm.brk, sm.nbrk, k - 1);  // first break >= k
    const uint32_t seg_end = (kb == kInf) ? kFar : T0 + kb;
    return min(seg_end, s + w);
}

// Pass 1: per-tile exit tables.  For candidate c (c < w: position T0+c;
// c == w: the end of the run crossing T0), tcode[t][c] is the exit code into
// tile t+1 and tcnt[t][c] the number of leaf starts visited inside tile t.
template <int KT>
__global__ __launch_bounds__(kThreads) void part_tables_kernel(
    const typename Key<KT>::raw* __restrict__ keys, uint32_t N, const uint64_t* __restrict__ offsets,
    uint32_t nseg, const uint32_t* __restrict__ tile_seg, uint32_t w, uint8_t* __restrict__ tcode,
    uint32_t* __restrict__ tcnt, TileRec* __restrict__ tile_rec, uint32_t* __restrict__ samp) {
    __shared__ PartShared<KT> sm;
    const uint32_t T0 = blockIdx.x * kPartTile;
    const uint32_t T1 = min(N, T0 + kPartTile);
    const uint32_t len = T1 - T0;
    const uint32_t W1 = w + 1;
    const int mode = tile_successors<KT>(keys, N, offsets, nseg, tile_seg, w, T0, T1, sm, samp);
    // The sample's stores wait until no barrier follows (a barrier would wait
    // for them).
    auto store_samples = [&]() {
        if (sizeof(typename Key<KT>::ukey) == 4 && samp) {
            const uint32_t m = threadIdx.x;
            if (m < (len + kSampleSpacing - 1) / kSampleSpacing) samp[T0 / kSampleSpacing + m] = sm.smp[m];
        }
    };
    {
        // the record the emit pass follows instead of reloading the keys
        TileRec* R = tile_rec + blockIdx.x;
        const uint32_t tid = threadIdx.x;
        if (tid == 0) {
            R->x0 = sm.x0;
            R->mode = (uint8_t)mode;
            R->t0 = sm.pt[0];
            R->nchg = (uint8_t)(mode == kTileWalk ? sm.nchg : 0u);
            R->nbrk = (uint8_t)(mode == kTileWalk ? sm.nbrk : 0u);
        }
        if (mode == kTileWalk) {
            if (tid < sm.nchg) {
                R->chg[tid] = sm.chg[tid];
                R->ctype[tid] = sm.pt[sm.chg[tid]];
            }
            if (tid < sm.nbrk) R->brk[tid] = sm.brk[tid];
        }
    }
    if (mode == kTileUniform) {
        // Entering at T0 + c (< T1): one leaf start, then past the window.
        // Entering at the crossing run's end: that end lies past the window.
        for (uint32_t c = threadIdx.x; c < W1; c += kThreads) {
            const bool via_run = (c == w) && sm.x0 == kFar;
            tcode[(size_t)blockIdx.x * W1 + c] = (uint8_t)w;
            tcnt[(size_t)blockIdx.x * W1 + c] = via_run ? 0u : 1u;
        }
        store_samples();
        return;
    }

    // Table mode: pointer jumping to the exits, counting visited positions.
    // One buffer: each round reads every position's next state into
    // registers, waits, then writes them back.  Walk mode follows each
    // candidate's chain below instead.
    const bool walk = (mode == kTileWalk);
    const bool jump = (mode == kTileTable);
    constexpr int kPJ = kPartTile / kThreads;  // positions per thread
    for (uint32_t i = threadIdx.x; jump && i < len; i += kThreads) sm.u.pj.ct[i] = 1;
    __syncthreads();
    for (int round = 0; jump && round < 16; ++round) {
        int any = 0;
        uint16_t na[kPJ], nc[kPJ];
#pragma unroll
        for (int q = 0; q < kPJ; ++q) {
            const uint32_t i = threadIdx.x + q * kThreads;
            if (i < len) {
                const uint16_t a = sm.u.pj.nx[i];
                na[q] = a;
                nc[q] = sm.u.pj.ct[i];
                if (!(a & kExitBit)) {
                    na[q] = sm.u.pj.nx[a];
                    nc[q] = (uint16_t)(nc[q] + sm.u.pj.ct[a]);
                    any |= !(na[q] & kExitBit);
                }
            }
        }
        __syncthreads();
#pragma unroll
        for (int q = 0; q < kPJ; ++q) {
            const uint32_t i = threadIdx.x + q * kThreads;
            if (i < len) {
                sm.u.pj.nx[i] = na[q];
                sm.u.pj.ct[i] = nc[q];
            }
        }
        if (!__syncthreads_or(any)) break;
    }

    for (uint32_t c = threadIdx.x; c < W1; c += kThreads) {
        uint32_t pos;
        bool valid = true;
        if (c < w) {
            pos = T0 + c;
        } else {
            pos = sm.x0;
            if (pos == kInf || (pos != kFar && pos < T0 + w)) valid = false;  // never entered this way
        }
        uint8_t code;
        uint32_t cnt;
        if (!valid) {
            pos = T0;  // filler: any well-defined entry
        }
        if (pos == kFar || pos >= T1) {
            code = (uint8_t)((pos != kFar && pos - T1 < w) ? (pos - T1) : w);
            cnt = 0;
        } else if (walk) {
            uint32_t s = pos;
            cnt = 0;
            while (s < T1) {
                ++cnt;
                s = walk_next<KT>(sm, T0, s, w);
            }
            code = (uint8_t)((s != kFar && s - T1 < w) ? (s - T1) : w);
        } else if (mode == kTileDense) {
            cnt = (T1 - pos + w - 1) / w;  // pos, pos + w, ... below T1
            code = (uint8_t)(pos + cnt * w - T1);
        } else {
            const uint16_t e = sm.u.pj.nx[pos - T0];
            code = (uint8_t)(e & 0xFF);
            cnt = sm.u.pj.ct[pos - T0];
        }
        tcode[(size_t)blockIdx.x * W1 + c] = code;
        tcnt[(size_t)blockIdx.x * W1 + c] = cnt;
    }
    store_samples();
}

// Up-sweep: compose groups of kScanGroup consecutive tables into one.
// Table k maps an entry code to (exit code, count); composing k then k+1
// gives c -> (E_{k+1}[E_k[c]], C_k[c] + C_{k+1}[E_k[c]]).
__global__ __launch_bounds__(kThreads) void compose_up_kernel(const uint8_t* __restrict__ code_in,
                                                               const uint32_t* __restrict__ cnt_in,
                                                               uint32_t ntab, uint32_t W1,
                                                               uint8_t* __restrict__ code_out,
                                                               uint32_t* __restrict__ cnt_out) {
    extern __shared__ unsigned char dyn[];
    uint32_t* scnt = reinterpret_cast<uint32_t*>(dyn);                        // [kScanGroup][W1]
    uint8_t* scode = reinterpret_cast<uint8_t*>(scnt + kScanGroup * W1);      // [kScanGroup][W1]
    const uint32_t base = blockIdx.x * kScanGroup;
    const uint32_t m = min((uint32_t)kScanGroup, ntab - base);
    for (uint32_t i = threadIdx.x; i < m * W1; i += kThreads) {
        scode[i] = code_in[(size_t)base * W1 + i];
        scnt[i] = cnt_in[(size_t)base * W1 + i];
    }
    __syncthreads();
    // In-place tree: at stride s, table i (i % 2s == 0) absorbs table i+s.
    for (uint32_t s = 1; s < m; s <<= 1) {
        const uint32_t npairs = (m + 2 * s - 1) / (2 * s);
        for (uint32_t x = threadIdx.x; x < npairs * W1; x += kThreads) {
            const uint32_t pr = x / W1, c = x % W1;
            const uint32_t a = pr * 2 * s, b = a + s;
            if (b < m) {
                const uint32_t e = scode[a * W1 + c];
                scnt[a * W1 + c] += scnt[b * W1 + e];
                scode[a * W1 + c] = scode[b * W1 + e];
            }
        }
        __syncthreads();
    }
    for (uint32_t c = threadIdx.x; c < W1; c += kThreads) {
        code_out[(size_t)blockIdx.x * W1 + c] = scode[c];
        cnt_out[(size_t)blockIdx.x * W1 + c] = scnt[c];
    }
}

// Down-sweep: given each group's entry code and leaf offset, walk its tables
// in order and record every table's entry code and offset.  At the top level
// (entry_in == nullptr) the single group is entered at position 0 with
// offset 0; at level 0 (final != nullptr) the last group also writes r and
// starts[r] = N.
__global__ __launch_bounds__(kThreads) void compose_down_kernel(
    const uint8_t* __restrict__ code_in, const uint32_t* __restrict__ cnt_in, uint32_t ntab, uint32_t W1,
    const uint8_t* __restrict__ entry_in, const uint32_t* __restrict__ off_in, uint8_t* __restrict__ entry_out,
    uint32_t* __restrict__ off_out, uint32_t* __restrict__ r_out, uint32_t* __restrict__ starts, uint32_t N,
    uint32_t rcap) {
    extern __shared__ unsigned char dyn[];
    uint32_t* scnt = reinterpret_cast<uint32_t*>(dyn);
    uint8_t* scode = reinterpret_cast<uint8_t*>(scnt + kScanGroup * W1);
    const uint32_t base = blockIdx.x * kScanGroup;
    const uint32_t m = min((uint32_t)kScanGroup, ntab - base);
    for (uint32_t i = threadIdx.x; i < m * W1; i += kThreads) {
        scode[i] = code_in[(size_t)base * W1 + i];
        scnt[i] = cnt_in[(size_t)base * W1 + i];
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        uint32_t e = entry_in ? entry_in[blockIdx.x] : 0;
        uint32_t off = off_in ? off_in[blockIdx.x] : 0;
        for (uint32_t k = 0; k < m; ++k) {
            entry_out[base + k] = (uint8_t)e;
            off_out[base + k] = off;
            off += scnt[k * W1 + e];
            e = scode[k * W1 + e];
        }
        if (r_out && base + m == ntab) {
            off = min(off, rcap);  // never past the leaf arrays
            *r_out = off;
            starts[off] = N;
        }
    }
}

// Pass 2: emit the leaf starts of each tile, entered at its true entry code.
// The chain points are marked by doubling: after round k the first 2^k
// points from the entry are marked and nx holds J^(2^k).
template <int KT>
__global__ __launch_bounds__(kThreads) void part_emit_kernel(
    const typename Key<KT>::raw* __restrict__ keys, uint32_t N, const uint64_t* __restrict__ offsets,
    uint32_t nseg, const uint32_t* __restrict__ tile_seg, uint32_t w, const uint8_t* __restrict__ entry,
    const uint32_t* __restrict__ offs, const uint32_t* __restrict__ tcnt, const TileRec* __restrict__ tile_rec,
    uint32_t* __restrict__ starts, uint32_t rcap) {
    __shared__ PartShared<KT> sm;
    const uint32_t T0 = blockIdx.x * kPartTile;
    const uint32_t T1 = min(N, T0 + kPartTile);
    const uint32_t len = T1 - T0;
    const uint32_t e = entry[blockIdx.x];
    const uint32_t tid = threadIdx.x;
    // No leaf starts in this tile (e.g. it lies inside one long run).
    if (tcnt[(size_t)blockIdx.x * (w + 1) + e] == 0) return;
    const TileRec* R = tile_rec + blockIdx.x;
    const int rmode = R->mode;
    if (rmode == kTileUniform) {
        // Inside one long run: the only leaf start is the entry itself.
        const uint32_t pos = (e < w) ? (T0 + e) : R->x0;
        if (tid == 0 && pos < T1) {
            const uint32_t rank = offs[blockIdx.x];
            if (rank < rcap) starts[rank] = pos;
        }
        return;
    }
    if (rmode == kTileDense) {
        // the chain steps by w from its entry: starts pos, pos + w, ...
        const uint32_t pos = (e < w) ? (T0 + e) : R->x0;
        if (pos >= T1) return;  // also kFar / kInf
        const uint32_t cnt = (T1 - pos + w - 1) / w;
        const uint32_t rank0 = offs[blockIdx.x];
        for (uint32_t q = tid; q < cnt; q += kThreads)
            if (rank0 + q < rcap) starts[rank0 + q] = pos + q * w;
        return;
    }
    int mode = kTileWalk;
    if (rmode == kTileWalk) {
        // Rebuild the window's pair types and lists from the record: a pair's
        // type is that of the last change at or before it (or of pair 0).
        const uint32_t nchg = R->nchg, nbrk = R->nbrk;
        if (tid < nchg) {
            sm.chg[tid] = R->chg[tid];
            sm.ctype[tid] = R->ctype[tid];
        }
        if (tid < nbrk) sm.brk[tid] = R->brk[tid];
        if (tid == 0) {
            sm.nchg = nchg;
            sm.nbrk = nbrk;
            sm.x0 = R->x0;
        }
        __syncthreads();
        const uint32_t WE = (uint32_t)min<uint64_t>((uint64_t)N, (uint64_t)T1 + w + 1);
        const uint32_t NPW = WE - T0 + 1;
        const uint32_t k0 = tid * kPairItems;
        uint32_t idx = 0;
        while (idx < nchg && sm.chg[idx] <= k0) ++idx;
        const uint8_t t0 = R->t0;
#pragma unroll
        for (int i = 0; i < kPairItems; ++i) {
            const uint32_t k = k0 + i;
            if (idx < nchg && sm.chg[idx] == k) ++idx;
            if (k < NPW) sm.pt[k] = idx ? sm.ctype[idx - 1] : t0;
        }
        __syncthreads();
    } else {
        mode = tile_successors<KT>(keys, N, offsets, nseg, tile_seg, w, T0, T1, sm);  // kTileTable again
    }
    uint32_t pos = (e < w) ? (T0 + e) : sm.x0;
    if (pos == kFar || pos == kInf || pos >= T1) return;  // the chain skips this tile
    if (mode == kTileWalk) {
        // one lane follows the chain; its points are consecutive leaf starts
        if (tid == 0) {
            uint32_t rank = offs[blockIdx.x];
            for (uint32_t s = pos; s < T1; s = walk_next<KT>(sm, T0, s, w)) {
                if (rank < rcap) starts[rank] = s;
                ++rank;
            }
        }
        return;
    }
    for (uint32_t i = threadIdx.x; i < len; i += kThreads) sm.u.em.mk[i] = (i == pos - T0);
    __syncthreads();
    constexpr int kPJ = kPartTile / kThreads;  // positions per thread
    for (int round = 0; round < 16; ++round) {
        // Mark the images of marked positions and read the doubled pointers;
        // a mark set during this phase and seen by another thread only adds
        // further points of the same chain.
        int any = 0;
        uint16_t na[kPJ];
#pragma unroll
        for (int q = 0; q < kPJ; ++q) {
            const uint32_t i = threadIdx.x + q * kThreads;
            if (i < len) {
                const uint16_t a = sm.u.em.nx[i];
                na[q] = a;
                if (!(a & kExitBit)) {
                    if (sm.u.em.mk[i]) sm.u.em.mk[a] = 1;
                    na[q] = sm.u.em.nx[a];
                    any |= !(na[q] & kExitBit);
                }
            }
        }
        __syncthreads();
#pragma unroll
        for (int q = 0; q < kPJ; ++q) {
            const uint32_t i = threadIdx.x + q * kThreads;
            if (i < len) sm.u.em.nx[i] = na[q];
        }
        // Once J^(2^(round+1)) leaves the tile from every position, the chain
        // from the entry has at most 2^(round+1) points, all marked by now.
        if (!__syncthreads_or(any)) break;
    }
    // Compact the marks in position order.
    uint32_t cnt = 0;
    const uint32_t i0 = threadIdx.x * kPartItems;
#pragma unroll
    for (int i = 0; i < kPartItems; ++i)
        if (i0 + i < len && sm.u.em.mk[i0 + i]) ++cnt;
    uint32_t rank = block_excl_sum(cnt, sm.sh, nullptr) + offs[blockIdx.x];
#pragma unroll
    for (int i = 0; i < kPartItems; ++i)
        if (i0 + i < len && sm.u.em.mk[i0 + i]) {
            if (rank < rcap) starts[rank] = T0 + i0 + i;
            ++rank;
        }
}

// ------------------------------------------------------------- host launch

// For every tile, the first offsets index whose value is >= T0 (a binary
// search per tile, all tiles at once).
__global__ __launch_bounds__(kThreads) void tile_seg_kernel(const uint64_t* __restrict__ offsets, uint32_t nseg,
                                                            uint32_t ntiles, uint32_t* __restrict__ tile_seg) {
    for (uint32_t t = blockIdx.x * kThreads + threadIdx.x; t < ntiles; t += gridDim.x * kThreads) {
        const uint64_t v = (uint64_t)t * kPartTile;
        uint32_t lo = 0, hi = nseg + 1;
        while (lo < hi) {
            const uint32_t m = (lo + hi) >> 1;
            if (offsets[m] < v) lo = m + 1; else hi = m;
        }
        tile_seg[t] = lo;
    }
}

template <int KT>
hipError_t launch_partition_t(const PartitionArgs& a, hipStream_t st) {
    using raw = typename Key<KT>::raw;
    const uint32_t nT = a.ntab[0];
    const uint32_t W1 = a.w + 1;
    if (a.nseg > 1)
        hipLaunchKernelGGL(tile_seg_kernel, dim3(std::min<uint32_t>((nT + kThreads - 1) / kThreads, 4096u)),
                           dim3(kThreads), 0, st, a.offsets, a.nseg, nT, a.tile_seg);
    hipLaunchKernelGGL(part_tables_kernel<KT>, dim3(nT), dim3(kThreads), 0, st, (const raw*)a.keys, a.N,
                       a.offsets, a.nseg, a.tile_seg, a.w, a.code[0], a.cnt[0], a.tile_rec, a.samp);
    const size_t lds = (size_t)kScanGroup * W1 * 5;
    for (int l = 0; l + 1 < a.levels; ++l)
        hipLaunchKernelGGL(compose_up_kernel, dim3(a.ntab[l + 1]), dim3(kThreads), lds, st, a.code[l], a.cnt[l],
                           a.ntab[l], W1, a.code[l + 1], a.cnt[l + 1]);
    for (int l = a.levels - 1; l >= 0; --l) {
        const bool top = (l == a.levels - 1);
        hipLaunchKernelGGL(compose_down_kernel, dim3(top ? 1 : a.ntab[l + 1]), dim3(kThreads), lds, st, a.code[l],
                           a.cnt[l], a.ntab[l], W1, top ? nullptr : a.entry[l + 1], top ? nullptr : a.offs[l + 1],
                           a.entry[l], a.offs[l], l == 0 ? a.r_dev : nullptr, a.starts, a.N, a.rmax);
    }
    hipLaunchKernelGGL(part_emit_kernel<KT>, dim3(nT), dim3(kThreads), 0, st, (const raw*)a.keys, a.N, a.offsets,
                       a.nseg, a.tile_seg, a.w, a.entry[0], a.offs[0], a.cnt[0], a.tile_rec, a.starts, a.rmax);
    return hipGetLastError();
}

hipError_t launch_partition(int kt, const PartitionArgs& a, hipStream_t st) {
    switch (kt) {
    case KT_I32: return launch_partition_t<KT_I32>(a, st);
    case KT_U32: return launch_partition_t<KT_U32>(a, st);
    case KT_I64: return launch_partition_t<KT_I64>(a, st);
    case KT_U64: return launch_partition_t<KT_U64>(a, st);
    case KT_F32: return launch_partition_t<KT_F32>(a, st);
    }
    return hipErrorInvalidValue;
}

}  // namespace ps
