// The L hash tables (hash tables of non-empty buckets, Sec. 2.2).
//
// A table is its n (key, id) pairs grouped by directory bin -- the top B bits
// of the 31-bit key -- with ids ascending inside a bin, plus the directory
// dir[b] = first position of bin b (dir[2^B] = n).  A lookup of key k scans
// bin k >> (31 - B) and keeps the entries whose key equals k: that is the
// bucket of k.  B is about log2(n) - 2, so a bin holds a handful of entries
// besides the bucket itself.
//
// Built in two stable passes per table (three for large n):
//   pass 1  global partition by the top 8 key bits into 256 "super-bins":
//           per-tile digit histograms, a per-table scan, and a scatter that
//           ranks each tile's keys stably with wave ballots and writes every
//           digit's run contiguously through an LDS reorder buffer;
//   pass 1b (large n) a stable split of every super-bin by S more key bits
//           into groups of a few thousand entries;
//   pass 2  one workgroup per (table, group): a reorder by the remaining
//           key bits in LDS, ids ascending per bin, written back
//           contiguously, which also yields the directory entries of the
//           group's bins.
// Scattered 4-byte stores are far slower than coalesced ones on this GPU, so
// every pass stages its output in LDS first.
// Ids are implicit in pass 1 (a point's index), so the keys written by the
// hash kernel are read twice and each table entry is written twice (three
// times with pass 1b).  Between the passes an entry takes 8 bytes (key, id)
// or, when the tables store 16-bit keys and pass 2 merges no groups, 6
// bytes: the 23 key bits below the super-bin digit with the id's low 9 bits
// above them, and the id's remaining bits as 16 bits (ids below 2^25).
#include <type_traits>

#include "common.h"

namespace fclsh {

namespace {

// pass 1 (tiles of the table, partitioned by the top kHiBits key bits)
constexpr int kP1NT = 512;                 // threads of the pass-1 scatter
constexpr int kP1Waves = kP1NT / 64;
constexpr int kP1Items = 16;               // entries per thread
constexpr int kP1Tile = kP1NT * kP1Items;  // entries per tile
constexpr int kHistNT = 256;
// pass 1b and pass 2 (one workgroup per super-bin or group)
constexpr int kNT = 512;                   // threads of the pass-2 kernels
constexpr int kWaves = kNT / 64;
constexpr int kItems = 16;                 // entries per thread
constexpr int kTile = kNT * kItems;        // 8192 entries: largest group reordered in LDS
constexpr int kFastItems = 9;              // entries per thread in the pass-2 group kernel
constexpr int kFastTile = kNT * kFastItems;  // 4608: largest group of the group kernel
constexpr int kRestBlocks = 1024;          // grid of the stable pass-2 kernel
constexpr int kHiBits = 8;
constexpr int kHiBins = 1 << kHiBits;
constexpr int kMaxLoBits = 11;
// 6-byte entries between the passes: id bits kept beside the key's low bits
constexpr int kPkIdLow = 32 - (31 - kHiBits);
constexpr uint32_t kPkKeyMask = (1u << (31 - kHiBits)) - 1u;

// A wave's LDS operations execute in issue order; this keeps the compiler from
// moving plain LDS accesses across the atomics between phases.
[[maybe_unused]] __device__ inline void wave_lds_order() {
    __asm__ volatile("" ::: "memory");
    __builtin_amdgcn_wave_barrier();
}

__device__ inline uint64_t lanemask_lt() {
    const int lane = threadIdx.x & 63;
    return lane ? (~0ull >> (64 - lane)) : 0ull;
}

// Lanes of the wave holding the same `bits`-bit digit as this lane (among the
// lanes with ok set), from one ballot per digit bit: a lane differs from this
// one if, for some bit, its ballot bit differs from this lane's bit.  The
// sign-extended bit (0 or all ones) serves both the ballot and the XOR.
// Four VALU instructions per bit: the bit field extract, the compare that
// makes the ballot, and one three-input bit operation (acc | (neg ^ ballot),
// truth table 0xde) per half of the mask.  Written with the builtins because
// the plain expressions compile to six (a second shift for the compare, and
// separate XORs and ORs).
// N rounds at once, bit-major, so that the compares of one round fill the
// wait between another round's compare and the reads of its ballot.
template <int N>
__device__ inline void same_digit_lanes(const uint32_t (&dg)[N], int bits, const bool (&ok)[N],
                                        uint64_t (&same)[N]) {
    uint32_t dlo[N], dhi[N];
#pragma unroll
    for (int k = 0; k < N; ++k) dlo[k] = dhi[k] = 0;
    for (int b = 0; b < bits; ++b) {
        int32_t neg[N];
        uint64_t bb[N];
#pragma unroll
        for (int k = 0; k < N; ++k) {
            neg[k] = __builtin_amdgcn_sbfe(int32_t(dg[k]), b, 1);
            bb[k] = __builtin_amdgcn_uicmp(uint32_t(neg[k]), 0u, 33);  // 33: not equal
        }
#pragma unroll
        for (int k = 0; k < N; ++k) {
            dlo[k] = __builtin_amdgcn_bitop3_b32(uint32_t(neg[k]), dlo[k], uint32_t(bb[k]), 0xde);
            dhi[k] = __builtin_amdgcn_bitop3_b32(uint32_t(neg[k]), dhi[k], uint32_t(bb[k] >> 32), 0xde);
        }
    }
#pragma unroll
    for (int k = 0; k < N; ++k) same[k] = __ballot(ok[k]) & ~((uint64_t(dhi[k]) << 32) | dlo[k]);
}

// Stable ranks of a wave's ITEMS rounds of 64 digits (round-major, then lane
// order): rank = number of earlier entries of this wave with the same digit.
// The lowest lane of each digit group adds the group size to the wave's
// counter with an LDS atomic that returns the previous value; the atomics of
// one wave execute in program order, so no round waits for the previous one.
// wcw must hold zeros for all digits on entry and ends as the wave histogram.
template <int ITEMS, int GRP, typename DigitOf, typename ValidOf>  // GRP: rounds with atomics in flight together
__device__ inline void wave_stable_ranks_of(DigitOf digit, ValidOf ok, int bits, uint32_t *wcw,
                                            uint32_t (&rank)[ITEMS]) {
    const uint64_t lt = lanemask_lt();
#pragma unroll
    for (int g0 = 0; g0 < ITEMS; g0 += GRP) {
        uint32_t before[GRP], lead[GRP], old[GRP];
#pragma unroll
        for (int k = 0; k < GRP; k += 2) {  // two rounds at a time
            if (g0 + k >= ITEMS) break;
            const bool two = k + 1 < GRP && g0 + k + 1 < ITEMS;
            const uint32_t dg[2] = {digit(g0 + k), two ? digit(g0 + k + 1) : 0u};
            const bool v[2] = {ok(g0 + k), two && ok(g0 + k + 1)};
            uint64_t same[2];
            same_digit_lanes<2>(dg, bits, v, same);
#pragma unroll
            for (int h = 0; h < 2; ++h) {
                if (h == 1 && !two) break;
                before[k + h] = uint32_t(__popcll(same[h] & lt));
                lead[k + h] = same[h] ? uint32_t(__builtin_ctzll(same[h])) : 0u;
                old[k + h] = (v[h] && before[k + h] == 0) ? atomicAdd(&wcw[dg[h]], uint32_t(__popcll(same[h]))) : 0u;
            }
        }
#pragma unroll
        for (int k = 0; k < GRP; ++k)
            if (g0 + k < ITEMS) rank[g0 + k] = __shfl(old[k], int(lead[k]), 64) + before[k];
    }
}

template <int ITEMS>
__device__ inline void wave_stable_ranks(const uint32_t (&dg)[ITEMS], const bool (&ok)[ITEMS], int bits,
                                         uint32_t *wcw, uint32_t (&rank)[ITEMS]) {
    wave_stable_ranks_of<ITEMS, (ITEMS < 8 ? ITEMS : 8)>([&](int it) { return dg[it]; },
                                                          [&](int it) { return ok[it]; }, bits, wcw, rank);
}

// Block-wide exclusive scan; *total gets the sum.
__device__ inline uint32_t block_scan_u32(uint32_t v, uint32_t *sh, uint32_t *total) {
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int nw = blockDim.x >> 6;
    uint32_t x = v;
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) {
        const uint32_t y = __shfl_up(x, o, 64);
        if (lane >= o) x += y;
    }
    if (lane == 63) sh[wave] = x;
    __syncthreads();
    if (threadIdx.x == 0) {
        uint32_t run = 0;
        for (int w = 0; w < nw; ++w) {
            const uint32_t c = sh[w];
            sh[w] = run;
            run += c;
        }
        sh[nw] = run;
    }
    __syncthreads();
    const uint32_t res = x - v + sh[wave];
    if (total) *total = sh[nw];
    __syncthreads();
    return res;
}

// Turns the per-wave digit histograms wc[w][d] into per-wave exclusive
// offsets and returns the per-digit totals in tot[d].
template <int NT>
__device__ inline void wave_offsets(uint32_t *wc, int R, uint32_t *tot) {
    for (int d = threadIdx.x; d < R; d += NT) {
        uint32_t run = 0;
        for (int w = 0; w < NT / 64; ++w) {
            const uint32_t c = wc[w * R + d];
            wc[w * R + d] = run;
            run += c;
        }
        tot[d] = run;
    }
}

// In place: cnt[d] := base + exclusive prefix of cnt over d < R.
template <int NT>
__device__ inline void digit_starts(uint32_t *cnt, int R, uint32_t base, uint32_t *sh) {
    const int per = (R + NT - 1) / NT;
    const int d0 = threadIdx.x * per;
    uint32_t s = 0;
    for (int k = 0; k < per; ++k)
        if (d0 + k < R) s += cnt[d0 + k];
    uint32_t run = block_scan_u32(s, sh, nullptr) + base;
    for (int k = 0; k < per; ++k)
        if (d0 + k < R) {
            const uint32_t c = cnt[d0 + k];
            cnt[d0 + k] = run;
            run += c;
        }
    __syncthreads();
}

// ---------------------------------------------------------------------------
// Pass 1
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(kHistNT) void p1_hist_kernel(const uint32_t *__restrict__ keys, int64_t n,
                                                          uint32_t *__restrict__ hist, int nblk) {
    constexpr int HW = kHistNT / 64;
    __shared__ uint32_t h[HW][kHiBins];
    const int T = blockIdx.y, blk = blockIdx.x, wave = threadIdx.x >> 6;
    for (int i = threadIdx.x; i < HW * kHiBins; i += kHistNT) (&h[0][0])[i] = 0;
    __syncthreads();
    const uint32_t *kp = keys + int64_t(T) * n;
    const int64_t beg = int64_t(blk) * kP1Tile;
    const int64_t end = min(n, beg + kP1Tile);
    constexpr int PER = kP1Tile / kHistNT;  // keys per thread
    if (end - beg == kP1Tile) {
        // full tile: issue all loads before the counting
        uint32_t k[PER];
#pragma unroll
        for (int j = 0; j < PER; ++j) k[j] = kp[beg + j * kHistNT + threadIdx.x];
#pragma unroll
        for (int j = 0; j < PER; ++j) atomicAdd(&h[wave][k[j] >> (31 - kHiBits)], 1u);
    } else {
        for (int64_t e = beg + threadIdx.x; e < end; e += kHistNT)
            atomicAdd(&h[wave][kp[e] >> (31 - kHiBits)], 1u);
    }
    __syncthreads();
    uint32_t c = 0;
    for (int w = 0; w < HW; ++w) c += h[w][threadIdx.x];
    hist[(int64_t(T) * nblk + blk) * kHiBins + threadIdx.x] = c;  // tile-major
}

// Per table: hist[T][blk][d] := start (within the table) of tile blk's run of
// digit d; bstart[T][d] = start of super-bin d, bstart[T][256] = n; also
// clears pass 2's two group counters.  (A
// "last block scans" fusion into the histogram kernel needs a device-scope
// release per block, which writes back the L2 of the XCD; it measured 20x
// slower than this separate launch.)
constexpr int kScanSeg = 4;  // tile segments per table in the scan (kHiBins threads each)

__global__ __launch_bounds__(kHiBins * kScanSeg) void p1_scan_kernel(uint32_t *__restrict__ hist, int nblk, int64_t n,
                                                                    uint32_t *__restrict__ bstart,
                                                                    uint32_t *__restrict__ rest_count) {
    __shared__ uint32_t segsum[kScanSeg][kHiBins];
    __shared__ uint32_t dbase[kHiBins];
    __shared__ uint32_t sh[kHiBins * kScanSeg / 64 + 1];
    const int T = blockIdx.x, d = threadIdx.x % kHiBins, seg = threadIdx.x / kHiBins;
    const int per = (nblk + kScanSeg - 1) / kScanSeg;
    const int b0 = min(nblk, seg * per), b1 = min(nblk, b0 + per);
    uint32_t *h = hist + int64_t(T) * nblk * kHiBins + d;
    // pass 1: this segment's count of digit d, 8 independent loads at a time
    uint32_t s = 0;
    int b = b0;
    for (; b + 8 <= b1; b += 8) {
        uint32_t c[8];
#pragma unroll
        for (int k = 0; k < 8; ++k) c[k] = h[int64_t(b + k) * kHiBins];
#pragma unroll
        for (int k = 0; k < 8; ++k) s += c[k];
    }
    for (; b < b1; ++b) s += h[int64_t(b) * kHiBins];
    segsum[seg][d] = s;
    __syncthreads();
    uint32_t pre = 0, tot = 0;  // digit d: earlier segments, all segments
    for (int k = 0; k < kScanSeg; ++k) {
        const uint32_t v = segsum[k][d];
        pre += k < seg ? v : 0u;
        tot += v;
    }
    // digit starts: exclusive scan over d of the digit totals (segment 0's
    // threads come first in thread order and carry them)
    const uint32_t ex = block_scan_u32(seg == 0 ? tot : 0u, sh, nullptr);
    if (seg == 0) dbase[d] = ex;
    __syncthreads();
    // pass 2: run starts of digit d in this segment's tiles
    uint32_t run = dbase[d] + pre;
    b = b0;
    for (; b + 8 <= b1; b += 8) {
        uint32_t c[8];
#pragma unroll
        for (int k = 0; k < 8; ++k) c[k] = h[int64_t(b + k) * kHiBins];
#pragma unroll
        for (int k = 0; k < 8; ++k) {
            h[int64_t(b + k) * kHiBins] = run;
            run += c[k];
        }
    }
    for (; b < b1; ++b) {
        const uint32_t c = h[int64_t(b) * kHiBins];
        h[int64_t(b) * kHiBins] = run;
        run += c;
    }
    if (seg == 0) bstart[int64_t(T) * (kHiBins + 1) + d] = dbase[d];
    if (threadIdx.x == 0) bstart[int64_t(T) * (kHiBins + 1) + kHiBins] = uint32_t(n);
    if (T == 0 && threadIdx.x < 2) rest_count[threadIdx.x] = 0;  // pass 2's counters start at zero
}


// One pass-1 output entry: 8 bytes (key, id) or, with PK, 6 bytes (the
// key's bits below the super-bin digit with the id's low bits above them;
// the id's high bits as 16 bits).
template <bool PK>
__device__ inline void p1_put(uint32_t *ok, void *oi, uint32_t o, uint32_t key, uint32_t id) {
    if constexpr (PK) {
        ok[o] = (key & kPkKeyMask) | (id << (32 - kPkIdLow));
        static_cast<uint16_t *>(oi)[o] = uint16_t(id >> kPkIdLow);
    } else {
        ok[o] = key;
        static_cast<uint32_t *>(oi)[o] = id;
    }
}

// (4 waves per SIMD, i.e. 2 workgroups per CU: the 6-byte form's stores
// would otherwise take it to 132 VGPRs and 1 workgroup.)
template <bool PK>
__global__ __launch_bounds__(kP1NT) __attribute__((amdgpu_waves_per_eu(4))) void p1_scatter_kernel(const uint32_t *__restrict__ keys, int64_t n,
                                                         const uint32_t *__restrict__ offs, int nblk,
                                                         int64_t nitems, uint32_t *__restrict__ okeys,
                                                         void *__restrict__ oids) {
    __shared__ uint32_t wc[kP1Waves * kHiBins];
    __shared__ uint32_t tot[kHiBins];
    __shared__ uint32_t gpos[kHiBins];
    __shared__ uint32_t sk[kP1Tile];
    __shared__ uint16_t si[kP1Tile];
    __shared__ uint32_t sh[kP1Waves + 1];

    const int64_t w = xcd_contiguous_item(blockIdx.x, gridDim.x);
    if (w >= nitems) return;  // padding of the grid to a multiple of kXcds
    const int T = int(w / nblk), blk = int(w % nblk);
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int64_t toff = int64_t(T) * n;
    const int64_t beg = int64_t(blk) * kP1Tile;
    const int cnt = int(min<int64_t>(kP1Tile, n - beg));
    for (int i = threadIdx.x; i < kP1Waves * kHiBins; i += kP1NT) wc[i] = 0;
    for (int d = threadIdx.x; d < kHiBins; d += kP1NT) gpos[d] = offs[(int64_t(T) * nblk + blk) * kHiBins + d];
    __syncthreads();

    uint32_t rk[kP1Items], dg[kP1Items], rank[kP1Items];
    bool ok[kP1Items];
    // every lane loads (the index clamped to the tile's last entry); entries
    // past the end are marked invalid and never used
    const uint32_t *kt = keys + toff + beg;
#pragma unroll
    for (int it = 0; it < kP1Items; ++it) {
        const int e = wave * (64 * kP1Items) + it * 64 + lane;
        ok[it] = e < cnt;
        rk[it] = kt[min(e, cnt - 1)];
        dg[it] = rk[it] >> (31 - kHiBits);
    }
    wave_stable_ranks<kP1Items>(dg, ok, kHiBits, wc + wave * kHiBins, rank);
    __syncthreads();
    wave_offsets<kP1NT>(wc, kHiBins, tot);
    __syncthreads();
    digit_starts<kP1NT>(tot, kHiBins, 0u, sh);  // tot := block-local start of each digit
#pragma unroll
    for (int it = 0; it < kP1Items; ++it) {
        if (ok[it]) {
            const uint32_t lp = tot[dg[it]] + wc[wave * kHiBins + dg[it]] + rank[it];
            sk[lp] = rk[it];
            si[lp] = uint16_t(wave * (64 * kP1Items) + it * 64 + lane);
        }
    }
    // gpos := table position of a digit's run minus its start in the tile,
    // so the entry at tile position j goes to gpos[d] + j (mod 2^32, < n)
    for (int d = threadIdx.x; d < kHiBins; d += kP1NT) gpos[d] -= tot[d];
    __syncthreads();
    uint32_t *okt = okeys + toff;
    void *oit = PK ? static_cast<void *>(static_cast<uint16_t *>(oids) + toff)
                   : static_cast<void *>(static_cast<uint32_t *>(oids) + toff);
    const uint32_t b32 = uint32_t(beg);
    if (cnt == kP1Tile) {
        // full tile: all LDS reads first, then the stores
        uint32_t kk[kP1Items], ii[kP1Items];
#pragma unroll
        for (int k = 0; k < kP1Items; ++k) {
            kk[k] = sk[k * kP1NT + threadIdx.x];
            ii[k] = si[k * kP1NT + threadIdx.x];
        }
#pragma unroll
        for (int k = 0; k < kP1Items; ++k) {
            const uint32_t o = gpos[kk[k] >> (31 - kHiBits)] + uint32_t(k * kP1NT + threadIdx.x);
            p1_put<PK>(okt, oit, o, kk[k], b32 + ii[k]);
        }
    } else {
        for (int j = threadIdx.x; j < cnt; j += kP1NT) {
            const uint32_t key = sk[j];
            const uint32_t o = gpos[key >> (31 - kHiBits)] + uint32_t(j);
            p1_put<PK>(okt, oit, o, key, b32 + si[j]);
        }
    }
}

// ---------------------------------------------------------------------------
// Pass 2: one workgroup per (table, group).
//
// A group of at most kFastTile entries (the usual case) is done by the group
// kernel, which loads it once and counts its bins with LDS atomics; the
// atomics also hand every entry a slot inside its bin, in arbitrary order.
// The bin counts, scanned, are the bin starts (the directory entries).
//
// Slot branch, when no bin holds over kMaxFastBin entries: keys and ids are
// placed in LDS by slot.  Then, walking the slots in order, each entry's
// final position is its bin start plus the number of ids in its bin smaller
// than its own (ids are distinct).  Neighbouring lanes hold neighbouring
// slots, so they read the same few bins (LDS broadcasts) and loop about as
// long as the largest of those bins; each writes its entry straight to its
// final place, which lies inside the few cache lines the wave covers.
//
// Ballot branch, when a bin is larger (clustered data): stable ranks from
// wave ballots in input order (passes 1 and 1b are stable, so input order is
// id order), per-wave digit counters, and an LDS reorder.
//
// With 16-bit stored keys both branches give way to ordered per-wave slots
// with a check of the id order (see p2_group); the two branches above are
// then its fallbacks.
//
// Either way the result equals the stable reorder exactly.  Groups over
// kFastTile entries go to a second kernel: the same ballot ranks over a tile
// of kTile entries, or for larger groups a histogram read first and a
// chunk-by-chunk scatter with running digit starts.
// ---------------------------------------------------------------------------
constexpr uint32_t kMaxFastBin = 48;

// Words of the group kernel's reorder region: two kFastTile buffers, which
// also hold the stable branch's per-wave digit counters.
__host__ __device__ constexpr int p2_region_a(int lo_bits) {
    return 2 * kFastTile > (kWaves << lo_bits) ? 2 * kFastTile : (kWaves << lo_bits);
}

// Pass 2 works on groups: the entries of a table that share their top gbits
// key bits (gbits = 8, or 8 + S after the pass-1b split), a contiguous run
// after the previous passes.  The final table keys are KT: uint32_t, or
// uint16_t when the key bits below the directory bin fit 16 bits (the bin,
// known from the directory, holds the rest), which saves 2 of pass 2's 16
// bytes per entry and of a query's bytes per bucket entry.
//
// PK: the input entries are the 6-byte form.  Their key word holds the key
// bits pass 2 uses (the bin digit below the group's bits and the stored low
// bits, all below the super-bin digit when no groups are merged) and the
// id's low bits on top, which the digit mask and the 16-bit store both leave
// out.
template <typename KT, bool PK>
struct P2Args {
    const uint32_t *kin;        // the group's input run (table offset applied)
    const void *vin;            // its ids: uint32, or with PK the id's high bits as uint16
    KT *okey;                   // the group's output run
    uint32_t *oid;
    uint32_t *dr;               // directory entries of the group's bins
    uint32_t count;             // entries in the group
    uint32_t bs;                // group start within the table
    int shift, lo_bits;
    uint32_t mask;
    bool fallback;  // tests: treat the id-order check as failed
    // the id word of input entry e, and the id from it and the entry's key
    // word k (apart, so that a thread's loads are all issued before any of
    // them is waited for)
    __device__ uint32_t id_word(uint32_t e) const {
        if constexpr (PK)
            return static_cast<const uint16_t *>(vin)[e];
        else
            return static_cast<const uint32_t *>(vin)[e];
    }
    __device__ uint32_t id_of(uint32_t w, uint32_t k) const {
        if constexpr (PK)
            return (w << kPkIdLow) | (k >> (32 - kPkIdLow));
        else
            return w;
    }
    __device__ uint32_t id(uint32_t e, uint32_t k) const { return id_of(id_word(e), k); }
};

// Block-wide maximum of one value per thread.
__device__ inline uint32_t block_max_u32(uint32_t v, uint32_t *sh) {
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v = max(v, uint32_t(__shfl_xor(v, o, 64)));
    if (lane == 0) sh[wave] = v;
    __syncthreads();
    uint32_t m = 0;
    for (int w = 0; w < kWaves; ++w) m = max(m, sh[w]);
    __syncthreads();
    return m;
}

// A group of at most kFastTile entries.  Entries are loaded wave-major (wave
// w holds a contiguous run of the group, ipw rounds of 64), which the stable
// branch needs and the fast branch does not mind.
// Returns kGroupSlot or kGroupBallot for the branch taken.  SLOT_ONLY: a
// group with a bin over kMaxFastBin is left untouched for the second kernel
// (kGroupLeft) instead of taking the ballot branch.
constexpr int kGroupLeft = 0, kGroupSlot = 1, kGroupBallot = 2;

// ANY_BIN (with SLOT_ONLY): the slot branch takes every group of at most
// kFastTile entries without looking at its bin sizes (its ranking is right
// for any bin, only slower on a large one), which saves a block reduction.
template <typename KT, bool PK, bool SLOT_ONLY, bool ANY_BIN = false>
__device__ int p2_group(const P2Args<KT, PK> &a, uint32_t *lds, uint32_t *sh) {
    const int R = 1 << a.lo_bits;
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    // region A: keys and ids in slot (fast) or final (stable) order; in the
    // stable branch first the per-wave digit counters [kWaves][R].
    //
    // With 16-bit stored keys (WS) the slot branch counts bins per wave.  A
    // wave's LDS atomics run in issue order, so its entries of a bin receive
    // slots in input order when the lanes of one atomic that hit the same
    // counter are served in lane order, which is what the hardware does.
    // The branch does not rely on it: it places every entry at bin start +
    // the bin's entries of earlier waves + its slot, checks that ids ascend
    // within every bin (input order is id order), and writes the group out
    // contiguously; a group where they do not falls back to the id walk
    // (bins of at most kMaxFastBin), the ballot branch, or in the slot-only
    // form to the second kernel.
    constexpr bool WS = sizeof(KT) == 2;
    uint32_t *bk = lds;
    uint32_t *bv = lds + kFastTile;
    uint32_t *cnt = lds + p2_region_a(a.lo_bits);  // R + 1 words: bin counts, then bin starts and the end
    for (int i = threadIdx.x; i < R; i += kNT) cnt[i] = 0;
    if constexpr (WS)
        for (int i = threadIdx.x; i < kWaves * R; i += kNT) lds[i] = 0;  // per-wave bin counters
    if (threadIdx.x == 0) cnt[R] = a.count;
    __syncthreads();
    const uint32_t ipw = (a.count + kNT - 1) / kNT;  // rounds per wave, at most kFastItems
    const uint32_t wbase = uint32_t(wave) * 64u * ipw + uint32_t(lane);
    const auto ok = [&](int it) { return uint32_t(it) < ipw && wbase + uint32_t(it) * 64u < a.count; };
    uint32_t rk[kFastItems], rv[kFastItems], pos[kFastItems];
#pragma unroll
    for (int it = 0; it < kFastItems; ++it) {
        const uint32_t e = wbase + uint32_t(it) * 64u;
        rk[it] = ok(it) ? a.kin[e] : 0u;
        rv[it] = ok(it) ? a.id_word(e) : 0u;
    }
#pragma unroll
    for (int it = 0; it < kFastItems; ++it) rv[it] = a.id_of(rv[it], rk[it]);
    if constexpr (WS) {
#pragma unroll
        for (int it = 0; it < kFastItems; ++it)
            pos[it] = ok(it) ? atomicAdd(&lds[wave * R + ((rk[it] >> a.shift) & a.mask)], 1u) : 0u;
        __syncthreads();
        // per bin: the per-wave counts become per-wave starts, the total its count
        for (int d = threadIdx.x; d < R; d += kNT) {
            uint32_t run = 0;
            for (int w = 0; w < kWaves; ++w) {
                const uint32_t c = lds[w * R + d];
                lds[w * R + d] = run;
                run += c;
            }
            cnt[d] = run;
        }
    } else {
#pragma unroll
        for (int it = 0; it < kFastItems; ++it)
            pos[it] = ok(it) ? atomicAdd(&cnt[(rk[it] >> a.shift) & a.mask], 1u) : 0u;
    }
    __syncthreads();
    bool fast = true;
    if constexpr (!ANY_BIN) {
        uint32_t mx = 0;
        for (int i = threadIdx.x; i < R; i += kNT) mx = max(mx, cnt[i]);
        fast = block_max_u32(mx, sh) <= kMaxFastBin;
    }
    // the slot walk: each entry's final place is its bin start plus the ids
    // of its bin smaller than its own (bk, bv hold the group by bin)
    const auto walk_out = [&]() {
        for (uint32_t j = threadIdx.x; j < a.count; j += kNT) {
            const uint32_t k = bk[j], v = bv[j];
            const uint32_t dg = (k >> a.shift) & a.mask;
            const uint32_t b0 = cnt[dg], b1 = cnt[dg + 1];
            // ids of the bin smaller than v: four independent reads per step
            uint32_t r = b0, q = b0;
            for (; q + 4 <= b1; q += 4) {
                const uint32_t x0 = bv[q], x1 = bv[q + 1], x2 = bv[q + 2], x3 = bv[q + 3];
                r += uint32_t(x0 < v) + uint32_t(x1 < v) + uint32_t(x2 < v) + uint32_t(x3 < v);
            }
            for (; q < b1; ++q) r += bv[q] < v ? 1u : 0u;
            a.okey[r] = KT(k);
            a.oid[r] = v;
        }
    };
    if constexpr (WS) {
        // every group: the per-wave slots, then the check of the id order
        digit_starts<kNT>(cnt, R, 0u, sh);  // ends with a barrier
        for (int i = threadIdx.x; i < R; i += kNT) a.dr[i] = a.bs + cnt[i];
#pragma unroll
        for (int it = 0; it < kFastItems; ++it)
            if (ok(it)) {
                const uint32_t d = (rk[it] >> a.shift) & a.mask;
                pos[it] += cnt[d] + lds[wave * R + d];  // bin start + the bin's entries in earlier waves
            }
        __syncthreads();  // the counters' space becomes the slot buffer
#pragma unroll
        for (int it = 0; it < kFastItems; ++it)
            if (ok(it)) {
                bk[pos[it]] = rk[it];
                bv[pos[it]] = rv[it];
            }
        __syncthreads();
        bool bad = false;
        for (uint32_t j = threadIdx.x + 1; j < a.count; j += kNT)
            bad |= ((bk[j] ^ bk[j - 1]) >> a.shift & a.mask) == 0 && bv[j - 1] > bv[j];
        if (!__syncthreads_or(bad || a.fallback)) {
            for (uint32_t j = threadIdx.x; j < a.count; j += kNT) {
                a.okey[j] = KT(bk[j]);
                a.oid[j] = bv[j];
            }
            return kGroupSlot;
        }
        if (SLOT_ONLY && !fast) return kGroupLeft;  // the second kernel redoes the group
        if (fast) {
            walk_out();
            return kGroupSlot;
        }
        for (int i = threadIdx.x; i < kWaves * R; i += kNT) lds[i] = 0;  // ballot counters
        __syncthreads();
    } else {
        if (SLOT_ONLY && !fast) return kGroupLeft;
        if (!fast) {
            for (int i = threadIdx.x; i < kWaves * R; i += kNT) lds[i] = 0;  // per-wave counters
        }
        digit_starts<kNT>(cnt, R, 0u, sh);  // ends with a barrier
        for (int i = threadIdx.x; i < R; i += kNT) a.dr[i] = a.bs + cnt[i];
        if (fast) {
#pragma unroll
            for (int it = 0; it < kFastItems; ++it)
                if (ok(it)) {
                    const uint32_t q = cnt[(rk[it] >> a.shift) & a.mask] + pos[it];
                    bk[q] = rk[it];
                    bv[q] = rv[it];
                }
            __syncthreads();
            walk_out();
            return kGroupSlot;
        }
    }
    // stable branch: input order is id order; rank = bin start + entries of
    // the bin in earlier waves + earlier entries of this wave
    const auto digit = [&](int it) { return (rk[it] >> a.shift) & a.mask; };
    wave_stable_ranks_of<kFastItems, 3>(digit, ok, a.lo_bits, lds + wave * R, pos);
    __syncthreads();
    for (int d = threadIdx.x; d < R; d += kNT) {
        uint32_t run = 0;
        for (int w = 0; w < kWaves; ++w) {
            const uint32_t c = lds[w * R + d];
            lds[w * R + d] = run;
            run += c;
        }
    }
    __syncthreads();
#pragma unroll
    for (int it = 0; it < kFastItems; ++it) pos[it] += cnt[digit(it)] + lds[wave * R + digit(it)];
    __syncthreads();  // the counters' space becomes the reorder buffer
#pragma unroll
    for (int it = 0; it < kFastItems; ++it)
        if (ok(it)) {
            bk[pos[it]] = rk[it];
            bv[pos[it]] = rv[it];
        }
    __syncthreads();
    for (uint32_t j = threadIdx.x; j < a.count; j += kNT) {
        a.okey[j] = KT(bk[j]);
        a.oid[j] = bv[j];
    }
    return kGroupBallot;
}

// Stable path for a group of at most kTile entries.
template <typename KT, bool PK>
__device__ void p2_stable_single(const P2Args<KT, PK> &a, uint32_t *lds, uint32_t *sh) {
    const int R = 1 << a.lo_bits;
    // region A (kTile*2 words): first the per-wave counters [kWaves][R], then
    // the reordered keys and ids; region B: start[R], tot[R]
    uint32_t *wc = lds;
    uint32_t *rkey = lds;
    uint32_t *rid = lds + kTile;
    uint32_t *start = lds + 2 * kTile;
    uint32_t *tot = start + R;
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    for (int i = threadIdx.x; i < kWaves * R; i += kNT) wc[i] = 0;
    __syncthreads();
    uint32_t rk[kItems], rv[kItems], dg[kItems], rank[kItems];
    bool ok[kItems];
#pragma unroll
    for (int it = 0; it < kItems; ++it) {
        const uint32_t e = uint32_t(wave * (64 * kItems) + it * 64 + lane);
        ok[it] = e < a.count;
        rk[it] = ok[it] ? a.kin[e] : 0u;
        rv[it] = ok[it] ? a.id_word(e) : 0u;
    }
#pragma unroll
    for (int it = 0; it < kItems; ++it) {
        rv[it] = a.id_of(rv[it], rk[it]);
        dg[it] = (rk[it] >> a.shift) & a.mask;
    }
    wave_stable_ranks<kItems>(dg, ok, a.lo_bits, wc + wave * R, rank);
    __syncthreads();
    wave_offsets<kNT>(wc, R, tot);
    __syncthreads();
    for (int i = threadIdx.x; i < R; i += kNT) start[i] = tot[i];
    __syncthreads();
    digit_starts<kNT>(start, R, 0u, sh);
    for (int i = threadIdx.x; i < R; i += kNT) a.dr[i] = a.bs + start[i];
#pragma unroll
    for (int it = 0; it < kItems; ++it)
        if (ok[it]) rank[it] += start[dg[it]] + wc[wave * R + dg[it]];
    __syncthreads();  // the counters' space becomes the reorder buffer
#pragma unroll
    for (int it = 0; it < kItems; ++it)
        if (ok[it]) {
            rkey[rank[it]] = rk[it];
            rid[rank[it]] = rv[it];
        }
    __syncthreads();
    for (uint32_t j = threadIdx.x; j < a.count; j += kNT) {
        a.okey[j] = KT(rkey[j]);
        a.oid[j] = rid[j];
    }
}

// Stable path for a group of more than kTile entries.
template <typename KT, bool PK>
__device__ void p2_stable_chunked(const P2Args<KT, PK> &a, uint32_t *lds, uint32_t *sh) {
    const int R = 1 << a.lo_bits;
    uint32_t *wc = lds;
    uint32_t *start = lds + 2 * kTile;
    uint32_t *tot = start + R;
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    for (int i = threadIdx.x; i < R; i += kNT) start[i] = 0;
    __syncthreads();
    for (uint32_t e = threadIdx.x; e < a.count; e += kNT) atomicAdd(&start[(a.kin[e] >> a.shift) & a.mask], 1u);
    __syncthreads();
    digit_starts<kNT>(start, R, 0u, sh);
    for (int i = threadIdx.x; i < R; i += kNT) a.dr[i] = a.bs + start[i];
    for (uint32_t c0 = 0; c0 < a.count; c0 += kTile) {
        for (int i = threadIdx.x; i < kWaves * R; i += kNT) wc[i] = 0;
        __syncthreads();
        uint32_t dg[kItems], rank[kItems];
        bool ok[kItems];
#pragma unroll
        for (int it = 0; it < kItems; ++it) {
            const uint32_t e = c0 + uint32_t(wave * (64 * kItems) + it * 64 + lane);
            ok[it] = e < a.count;
            dg[it] = ok[it] ? (a.kin[e] >> a.shift) & a.mask : 0u;
        }
        wave_stable_ranks<kItems>(dg, ok, a.lo_bits, wc + wave * R, rank);
        __syncthreads();
        wave_offsets<kNT>(wc, R, tot);
        __syncthreads();
#pragma unroll
        for (int it = 0; it < kItems; ++it)
            if (ok[it]) {
                const uint32_t e = c0 + uint32_t(wave * (64 * kItems) + it * 64 + lane);
                const uint32_t dst = start[dg[it]] + wc[wave * R + dg[it]] + rank[it];
                const uint32_t k = a.kin[e];
                a.okey[dst] = KT(k);
                a.oid[dst] = a.id(e, k);
            }
        __syncthreads();
        for (int d = threadIdx.x; d < R; d += kNT) start[d] += tot[d];
        __syncthreads();
    }
}

// Pass-2 group g is groups [g << gk, (g + 1) << gk) of the earlier passes:
// gk > 0 merges small neighbouring groups (their keys already in order), and
// gbits + lo_bits = dir_bits either way.
template <typename KT, bool PK>
__device__ inline P2Args<KT, PK> p2_args(const uint32_t *ikeys, const void *iids, int64_t n,
                                         const uint32_t *gstart, int gbits, int lo_bits, int gk, KT *tkeys,
                                         uint32_t *tids, uint32_t *dir, int T, int g, bool fallback = false) {
    const int64_t toff = int64_t(T) * n;
    // group starts per table: 2^(gbits + gk) + 1 (<= 4097), so the index
    // fits 32 bits and stays in scalar registers (a 64-bit product lands in
    // vector registers, and the block-uniform loop exits of the group kernel
    // then become exec-masked)
    const uint32_t gs = (1u << (gbits + gk)) + 1u;
    const uint32_t gi = uint32_t(T) * gs + (uint32_t(g) << gk);
    const uint32_t bs = gstart[gi];
    const uint32_t be = gstart[gi + (1u << gk)];
    P2Args<KT, PK> a;
    a.kin = ikeys + toff + bs;
    if constexpr (PK)
        a.vin = static_cast<const uint16_t *>(iids) + toff + bs;
    else
        a.vin = static_cast<const uint32_t *>(iids) + toff + bs;
    a.okey = tkeys + toff + bs;
    a.oid = tids + toff + bs;
    a.dr = dir + int64_t(T) * ((int64_t(1) << (gbits + lo_bits)) + 1) + (int64_t(g) << lo_bits);
    a.count = be - bs;
    a.bs = bs;
    a.lo_bits = lo_bits;
    a.shift = 31 - gbits - lo_bits;
    a.mask = (1u << lo_bits) - 1u;
    a.fallback = fallback;
    return a;
}

// Pass 2, group kernel over every (table, group); groups over kFastTile
// entries (and, in the slot-only form, groups with a large bin) are appended
// to rest[] for p2_rest_kernel.  counts[0] = listed groups, counts[1] =
// groups that took the ballot branch.  The slot-only form (51 VGPRs, 4
// workgroups per CU) is chosen for a rebuild when the previous build sent
// at most 1 % of the groups off the slot branch, with ANY_BIN (60 VGPRs)
// when it sent none; the full form needs 68 VGPRs (3 per CU).
// (iids and tids may be the same array: the ids are then reordered in place,
// each group reading its whole run into registers before writing it.)
template <typename KT, bool PK, bool SLOT_ONLY, bool ANY_BIN = false>
__global__ __launch_bounds__(kNT, SLOT_ONLY ? 8 : 6) void p2_fast_kernel(
    const uint32_t *__restrict__ ikeys, const void *iids, int64_t n, const uint32_t *__restrict__ gstart,
    int gbits, int lo_bits, int gk, KT *__restrict__ tkeys, uint32_t *tids, uint32_t *__restrict__ dir,
    uint32_t *__restrict__ rest, uint32_t *__restrict__ counts, int64_t nitems, int fallback) {
    extern __shared__ __align__(16) uint32_t lds[];
    __shared__ uint32_t sh[kWaves + 1];
    const int64_t w = xcd_contiguous_item(blockIdx.x, gridDim.x);
    if (w >= nitems) return;  // grid padding
    const int T = int(w >> gbits), g = int(w & ((int64_t(1) << gbits) - 1));
    if (g == (1 << gbits) - 1 && threadIdx.x == 0)
        dir[int64_t(T) * ((int64_t(1) << (gbits + lo_bits)) + 1) + (int64_t(1) << (gbits + lo_bits))] = uint32_t(n);
    const P2Args<KT, PK> a =
        p2_args<KT, PK>(ikeys, iids, n, gstart, gbits, lo_bits, gk, tkeys, tids, dir, T, g, fallback != 0);
    const int how = a.count <= uint32_t(kFastTile) ? p2_group<KT, PK, SLOT_ONLY, ANY_BIN>(a, lds, sh) : kGroupLeft;
    if (threadIdx.x == 0) {
        if (how == kGroupLeft) rest[atomicAdd(counts, 1u)] = uint32_t(w);
        if (how == kGroupBallot) atomicAdd(counts + 1, 1u);
    }
}

// Pass 2, stable path for the groups the group kernel left: a fixed grid
// works through the list (empty on uniform keys).  When the input ids are the
// output id array (after the pass-1b split), a group taking the chunked
// path first copies its ids to spare, which that path then reads.
template <typename KT, bool PK>
__global__ __launch_bounds__(kNT, 4) void p2_rest_kernel(const uint32_t *__restrict__ ikeys, const void *iids,
                                                         int64_t n, const uint32_t *__restrict__ gstart, int gbits,
                                                         int lo_bits, int gk, KT *__restrict__ tkeys,
                                                         uint32_t *tids,
                                                         uint32_t *__restrict__ dir, const uint32_t *__restrict__ rest,
                                                         const uint32_t *__restrict__ rest_count,
                                                         uint32_t *__restrict__ spare) {
    extern __shared__ __align__(16) uint32_t lds[];
    __shared__ uint32_t sh[kWaves + 1];
    const uint32_t nrest = *rest_count;
    for (uint32_t i = blockIdx.x; i < nrest; i += gridDim.x) {
        const int64_t w = rest[i];
        const int T = int(w >> gbits), g = int(w & ((int64_t(1) << gbits) - 1));
        P2Args<KT, PK> a = p2_args<KT, PK>(ikeys, iids, n, gstart, gbits, lo_bits, gk, tkeys, tids, dir, T, g);
        if (a.count > uint32_t(kTile)) {
            if constexpr (!PK) {
                if (iids == tids) {
                    uint32_t *copy = spare + int64_t(T) * n + a.bs;
                    for (uint32_t e = threadIdx.x; e < a.count; e += kNT) copy[e] = a.id(e, 0u);
                    __syncthreads();
                    a.vin = copy;
                }
            }
            p2_stable_chunked<KT, PK>(a, lds, sh);
        } else {
            p2_stable_single<KT, PK>(a, lds, sh);
        }
        __syncthreads();  // LDS reuse by the next item
    }
}

// Pass 1b, for large tables: one workgroup per (table, super-bin) splits the
// super-bin stably by the next sbits key bits into 2^sbits groups, so that
// pass 2 sees groups of a few thousand entries.  A histogram of the
// sub-digits gives the group starts (gstart, the pass-2 layout); the
// super-bin is then moved chunk by chunk (wave-ballot ranks, LDS reorder)
// with running group offsets, each sub-digit's run written contiguously.
// Chunks are 4096 entries (8 per thread; 80 VGPRs and 33 KB of LDS: 3
// workgroups per CU) up to 8 sub-digits, and 8192 (2 per CU) for 16, which
// keeps every chunk's runs at 512 entries or more.
constexpr int kMaxSplitBits = 4;

// PK: 6-byte entries (pass 1's packed form, kept): the split reads its
// sub-digit from the key word's low bits and moves the 16-bit id word along
// unchanged; the id itself is assembled only by pass 2.
template <int ITEMS, bool PK>
__global__ __launch_bounds__(kNT, ITEMS <= 8 ? 6 : 4) void p1b_split_kernel(const uint32_t *__restrict__ ikeys,
                                                           const void *__restrict__ iids, int64_t n,
                                                           const uint32_t *__restrict__ bstart, int sbits,
                                                           uint32_t *__restrict__ okeys, void *__restrict__ oids,
                                                           uint32_t *__restrict__ gstart, int64_t nitems) {
    using VT = typename std::conditional<PK, uint16_t, uint32_t>::type;
    constexpr int MS = 1 << kMaxSplitBits;
    constexpr int CHUNK = kNT * ITEMS;
    __shared__ uint32_t sk[CHUNK];
    __shared__ uint32_t sv[CHUNK];
    __shared__ uint32_t wc[kWaves * MS];
    __shared__ uint32_t cnt[MS], run[MS], ctot[MS], cst[MS];
    const int64_t w = xcd_contiguous_item(blockIdx.x, gridDim.x);
    if (w >= nitems) return;  // grid padding
    const int T = int(w / kHiBins), sb = int(w % kHiBins);
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int SB = 1 << sbits;
    const int shift = 31 - kHiBits - sbits;
    const uint32_t mask = uint32_t(SB - 1);
    const uint32_t bs = bstart[int64_t(T) * (kHiBins + 1) + sb];
    const uint32_t count = bstart[int64_t(T) * (kHiBins + 1) + sb + 1] - bs;
    const int64_t off = int64_t(T) * n + bs;
    const uint32_t *kin = ikeys + off;
    const VT *vin = static_cast<const VT *>(iids) + off;
    uint32_t *okey = okeys + off;
    VT *oid = static_cast<VT *>(oids) + off;
    if (threadIdx.x < MS) cnt[threadIdx.x] = 0;
    __syncthreads();
    {
        // sub-digit histogram, 16 independent loads in flight per thread
        uint32_t e = threadIdx.x;
        for (; e + 15u * kNT < count; e += 16u * kNT) {
            uint32_t kk[16];
#pragma unroll
            for (int u = 0; u < 16; ++u) kk[u] = kin[e + uint32_t(u) * kNT];
#pragma unroll
            for (int u = 0; u < 16; ++u) atomicAdd(&cnt[(kk[u] >> shift) & mask], 1u);
        }
        for (; e < count; e += kNT) atomicAdd(&cnt[(kin[e] >> shift) & mask], 1u);
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        const int64_t gs = (int64_t(kHiBins) << sbits) + 1;
        uint32_t acc = 0;
        for (int d = 0; d < SB; ++d) {
            gstart[int64_t(T) * gs + (int64_t(sb) << sbits) + d] = bs + acc;
            run[d] = acc;
            acc += cnt[d];
        }
        if (sb == kHiBins - 1) gstart[int64_t(T) * gs + gs - 1] = uint32_t(n);
    }
    __syncthreads();
    for (uint32_t c0 = 0; c0 < count; c0 += CHUNK) {
        for (int i = threadIdx.x; i < kWaves * SB; i += kNT) wc[i] = 0;
        __syncthreads();
        uint32_t rk[ITEMS], rv[ITEMS], dg[ITEMS], rank[ITEMS];
        bool ok[ITEMS];
#pragma unroll
        for (int it = 0; it < ITEMS; ++it) {
            const uint32_t e = c0 + uint32_t(wave * (64 * ITEMS) + it * 64 + lane);
            ok[it] = e < count;
            rk[it] = ok[it] ? kin[e] : 0u;
            rv[it] = ok[it] ? vin[e] : 0u;
            dg[it] = (rk[it] >> shift) & mask;
        }
        wave_stable_ranks<ITEMS>(dg, ok, sbits, wc + wave * SB, rank);
        __syncthreads();
        wave_offsets<kNT>(wc, SB, ctot);
        __syncthreads();
        if (threadIdx.x == 0) {
            uint32_t acc = 0;
            for (int d = 0; d < SB; ++d) {
                cst[d] = acc;
                acc += ctot[d];
            }
        }
        __syncthreads();
#pragma unroll
        for (int it = 0; it < ITEMS; ++it)
            if (ok[it]) {
                const uint32_t lp = cst[dg[it]] + wc[wave * SB + dg[it]] + rank[it];
                sk[lp] = rk[it];
                sv[lp] = rv[it];
            }
        __syncthreads();
        const uint32_t chunk = min(uint32_t(CHUNK), count - c0);
        if (chunk == uint32_t(CHUNK)) {
            // full chunk: all LDS reads first, then the stores
            uint32_t kk[ITEMS], vv[ITEMS];
#pragma unroll
            for (int k = 0; k < ITEMS; ++k) {
                kk[k] = sk[k * kNT + threadIdx.x];
                vv[k] = sv[k * kNT + threadIdx.x];
            }
#pragma unroll
            for (int k = 0; k < ITEMS; ++k) {
                const uint32_t d = (kk[k] >> shift) & mask;
                const uint32_t dst = run[d] + (uint32_t(k * kNT) + threadIdx.x - cst[d]);
                okey[dst] = kk[k];
                oid[dst] = VT(vv[k]);
            }
        } else {
            for (uint32_t j = threadIdx.x; j < chunk; j += kNT) {
                const uint32_t key = sk[j];
                const uint32_t d = (key >> shift) & mask;
                const uint32_t dst = run[d] + (j - cst[d]);
                okey[dst] = key;
                oid[dst] = VT(sv[j]);
            }
        }
        __syncthreads();
        if (threadIdx.x < SB) run[threadIdx.x] += ctot[threadIdx.x];
        __syncthreads();
    }
}

}  // namespace

int table_dir_bits(int64_t n) {
    int b = 0;
    while ((int64_t(1) << (b + 1)) <= n) ++b;  // floor(log2 n)
    b -= 2;
    if (b < kHiBits) b = kHiBits;
    if (b > kHiBits + kMaxLoBits) b = kHiBits + kMaxLoBits;
    return b;
}

// Extra key bits by which pass 1b splits each super-bin, so that pass 2's
// groups average at most 4096 entries (0 up to about a million points).
int table_split_bits(int64_t n, int dir_bits) {
    int sb = 0;
    while (sb < kMaxSplitBits && (n >> (kHiBits + sb)) > 4096) ++sb;
    return std::min(sb, dir_bits - kHiBits);
}

// Groups that pass 2 merges into one (as a shift), for small tables: the
// merged groups average at most 2048 entries, their bin count stays within
// 2^9 (so the group kernel's LDS is what it is unmerged) and at least 8
// groups remain per table.
int table_merge_bits(int64_t n, int dir_bits) {
    const int gbits = kHiBits + table_split_bits(n, dir_bits);
    int gk = 0;
    while ((n >> (gbits - gk - 1)) <= 2048 && dir_bits - gbits + gk + 1 <= 9 && gbits - gk - 1 >= 3) ++gk;
    return gk;
}

// tile histograms [L][tiles][256], super-bin starts [L][257], group starts
// [L][(256 << S) + 1] (S > 0 only), the count of groups left to the stable
// pass-2 kernel, and the list of those groups [L][256 << S]
size_t table_build_scratch_bytes(int64_t L, int64_t n, int dir_bits) {
    const int64_t nblk = (n + kP1Tile - 1) / kP1Tile;
    const int S = table_split_bits(n, dir_bits);
    const size_t groups = size_t(kHiBins) << S;
    return 4 * (size_t(L) * nblk * kHiBins + size_t(L) * (kHiBins + 1) + (S ? size_t(L) * (groups + 1) : 0) + 2 +
                size_t(L) * groups);
}

const uint32_t *table_build_counts(const uint32_t *scratch, int64_t L, int64_t n, int dir_bits) {
    const int64_t nblk = (n + kP1Tile - 1) / kP1Tile;
    const int S = table_split_bits(n, dir_bits);
    return scratch + size_t(L) * nblk * kHiBins + size_t(L) * (kHiBins + 1) +
           (S ? size_t(L) * ((size_t(kHiBins) << S) + 1) : 0);
}

namespace {

template <typename KT, bool PK>
fclsh_status launch_pass2(const uint32_t *p2k, const void *p2v, int64_t L, int64_t n, const uint32_t *gstart,
                          int gbits2, int lo_bits2, int gk, KT *tkeys, uint32_t *tids, uint32_t *dir, uint32_t *rest,
                          uint32_t *rest_count, uint32_t *tmpv, BuildMode mode, bool fallback, hipStream_t st,
                          hipEvent_t *marks) {
    const int fb = fallback ? 1 : 0;
    const size_t lds2 = (size_t(2) * kTile + 2 * (size_t(1) << lo_bits2)) * 4;
    const size_t lds_fast = (size_t(p2_region_a(lo_bits2)) + (size_t(1) << lo_bits2) + 1) * 4;
    const int64_t nitems2 = int64_t(L) << gbits2;  // (table, group) items, a multiple of kXcds
    if (mode == BuildMode::kSlotAll)
        hipLaunchKernelGGL(HIP_KERNEL_NAME(p2_fast_kernel<KT, PK, true, true>), dim3(unsigned(nitems2)), dim3(kNT),
                           lds_fast, st, p2k, p2v, n, gstart, gbits2, lo_bits2, gk, tkeys, tids, dir, rest, rest_count,
                           nitems2, fb);
    else if (mode == BuildMode::kSlotOnly)
        hipLaunchKernelGGL(HIP_KERNEL_NAME(p2_fast_kernel<KT, PK, true>), dim3(unsigned(nitems2)), dim3(kNT), lds_fast, st,
                           p2k, p2v, n, gstart, gbits2, lo_bits2, gk, tkeys, tids, dir, rest, rest_count, nitems2, fb);
    else
        hipLaunchKernelGGL(HIP_KERNEL_NAME(p2_fast_kernel<KT, PK, false>), dim3(unsigned(nitems2)), dim3(kNT), lds_fast,
                           st, p2k, p2v, n, gstart, gbits2, lo_bits2, gk, tkeys, tids, dir, rest, rest_count, nitems2,
                           fb);
    FCLSH_HIP(hipGetLastError());
    if (marks) FCLSH_HIP(hipEventRecord(marks[4], st));
    hipLaunchKernelGGL(HIP_KERNEL_NAME(p2_rest_kernel<KT, PK>), dim3(unsigned(std::min<int64_t>(nitems2, kRestBlocks))), dim3(kNT), lds2,
                       st, p2k, p2v, n, gstart, gbits2, lo_bits2, gk, tkeys, tids, dir, rest, rest_count, tmpv);
    FCLSH_HIP(hipGetLastError());
    if (marks) FCLSH_HIP(hipEventRecord(marks[5], st));
    return FCLSH_OK;
}

}  // namespace

int table_key_bytes(int dir_bits) { return 31 - dir_bits <= 16 ? 2 : 4; }

bool table_packed_pass1(int64_t n, int dir_bits) {
    return table_key_bytes(dir_bits) == 2 && table_merge_bits(n, dir_bits) == 0 && n <= (int64_t(1) << (kPkIdLow + 16));
}

namespace {

// Whole keys of tables [T0, T1) from 16-bit stored keys: a thread per entry
// finds its bin by a binary search of the table's directory (the largest b
// with dir[b] <= j) and writes (b << (31 - dir_bits)) | low.  The work is
// n log 2^dir_bits per table whatever the bin sizes.
__global__ void expand_keys_kernel(const uint16_t *__restrict__ tk, const uint32_t *__restrict__ dir, int64_t n,
                                   int dir_bits, int T0, int64_t ntab, uint32_t *__restrict__ out) {
    const uint32_t nb = 1u << dir_bits;
    for (int64_t g = int64_t(blockIdx.x) * blockDim.x + threadIdx.x; g < ntab * n;
         g += int64_t(gridDim.x) * blockDim.x) {
        const int64_t t = g / n, j = g - t * n;
        const int64_t T = T0 + t;
        const uint32_t *dr = dir + T * (int64_t(nb) + 1);
        uint32_t lo = 0, hi = nb;  // dr[lo] <= j < dr[hi] (dr[0] = 0, dr[nb] = n)
        while (hi - lo > 1) {
            const uint32_t mid = (lo + hi) >> 1;
            if (dr[mid] <= uint32_t(j))
                lo = mid;
            else
                hi = mid;
        }
        out[g] = (lo << (31 - dir_bits)) | tk[T * n + j];
    }
}

}  // namespace

fclsh_status expand_table_keys(const void *tkeys, int key_bytes, const uint32_t *dir, int64_t n, int dir_bits, int T0,
                               int T1, uint32_t *out, hipStream_t st) {
    const int64_t ntab = T1 - T0;
    if (ntab <= 0) return FCLSH_OK;
    if (key_bytes == 4) {
        FCLSH_HIP(hipMemcpyAsync(out, static_cast<const uint32_t *>(tkeys) + int64_t(T0) * n, size_t(ntab * n) * 4,
                                 hipMemcpyDeviceToDevice, st));
        return FCLSH_OK;
    }
    const int64_t work = ntab * n;
    hipLaunchKernelGGL(expand_keys_kernel, dim3(unsigned(std::min<int64_t>((work + 255) / 256, 1 << 16))), dim3(256), 0,
                       st, static_cast<const uint16_t *>(tkeys), dir, n, dir_bits, T0, ntab, out);
    FCLSH_HIP(hipGetLastError());
    return FCLSH_OK;
}

fclsh_status build_tables_2pass(uint32_t *keys, int64_t L, int64_t n, int dir_bits, uint32_t *tmpk, uint32_t *tmpv,
                                uint32_t *scratch, void *tkeys, uint32_t *tids, uint32_t *dir, BuildMode mode,
                                bool p2_fallback, hipStream_t st, hipEvent_t *marks) {
    if (L == 0 || n == 0) return FCLSH_OK;
    if (L > 65535) return fail(FCLSH_EUNSUPPORTED, "too many tables");
    if (dir_bits < kHiBits || dir_bits > kHiBits + kMaxLoBits) return fail(FCLSH_EINVAL, "bad directory bits");
    const int nblk = int((n + kP1Tile - 1) / kP1Tile);
    const int S = table_split_bits(n, dir_bits);
    const int gk = table_merge_bits(n, dir_bits);
    const int gbits = kHiBits + S, lo_bits = dir_bits - gbits;  // groups of passes 1 and 1b
    const int gbits2 = gbits - gk, lo_bits2 = lo_bits + gk;     // pass 2's groups
    uint32_t *hist = scratch;
    uint32_t *bstart = hist + size_t(L) * nblk * kHiBins;
    uint32_t *gstart = S ? bstart + size_t(L) * (kHiBins + 1) : bstart;
    uint32_t *rest_count = S ? gstart + size_t(L) * ((size_t(kHiBins) << S) + 1) : bstart + size_t(L) * (kHiBins + 1);
    uint32_t *rest = rest_count + 2;
    hipLaunchKernelGGL(p1_hist_kernel, dim3(nblk, unsigned(L)), dim3(kHistNT), 0, st, keys, n, hist, nblk);
    FCLSH_HIP(hipGetLastError());
    if (marks) FCLSH_HIP(hipEventRecord(marks[0], st));
    hipLaunchKernelGGL(p1_scan_kernel, dim3(unsigned(L)), dim3(kHiBins * kScanSeg), 0, st, hist, nblk, n, bstart,
                       rest_count);
    FCLSH_HIP(hipGetLastError());
    if (marks) FCLSH_HIP(hipEventRecord(marks[1], st));
    const int64_t nitems = int64_t(nblk) * L;
    const int64_t grid1 = xcd_grid(nitems);
    if (grid1 > 0x7FFFFFFF) return fail(FCLSH_EUNSUPPORTED, "too many table tiles");
    // 6-byte entries between the passes when the tables store 16-bit keys
    // and pass 2 merges no groups
    const bool packed = table_packed_pass1(n, dir_bits);
    if (packed)
        hipLaunchKernelGGL(p1_scatter_kernel<true>, dim3(unsigned(grid1)), dim3(kP1NT), 0, st, keys, n, hist, nblk,
                           nitems, tmpk, static_cast<void *>(tmpv));
    else
        hipLaunchKernelGGL(p1_scatter_kernel<false>, dim3(unsigned(grid1)), dim3(kP1NT), 0, st, keys, n, hist, nblk,
                           nitems, tmpk, static_cast<void *>(tmpv));
    FCLSH_HIP(hipGetLastError());
    if (marks) FCLSH_HIP(hipEventRecord(marks[2], st));
    // pass 2 input: the pass-1 output, or after the split the hash-key buffer
    // (keys) and the table id array (ids reordered in place); with 6-byte
    // entries the split's 16-bit id words go to the second half of tmpv
    const uint32_t *p2k = tmpk;
    const void *p2v = tmpv;
    if (S) {
        const int64_t nsb = int64_t(kHiBins) * L;
        void *sv = packed ? static_cast<void *>(reinterpret_cast<uint16_t *>(tmpv) + L * n) : static_cast<void *>(tids);
        if (S <= 3 && packed)
            hipLaunchKernelGGL(HIP_KERNEL_NAME(p1b_split_kernel<8, true>), dim3(unsigned(nsb)), dim3(kNT), 0, st, tmpk,
                               tmpv, n, bstart, S, keys, sv, gstart, nsb);
        else if (S <= 3)
            hipLaunchKernelGGL(HIP_KERNEL_NAME(p1b_split_kernel<8, false>), dim3(unsigned(nsb)), dim3(kNT), 0, st,
                               tmpk, tmpv, n, bstart, S, keys, sv, gstart, nsb);
        else if (packed)
            hipLaunchKernelGGL(HIP_KERNEL_NAME(p1b_split_kernel<16, true>), dim3(unsigned(nsb)), dim3(kNT), 0, st,
                               tmpk, tmpv, n, bstart, S, keys, sv, gstart, nsb);
        else
            hipLaunchKernelGGL(HIP_KERNEL_NAME(p1b_split_kernel<16, false>), dim3(unsigned(nsb)), dim3(kNT), 0, st,
                               tmpk, tmpv, n, bstart, S, keys, sv, gstart, nsb);
        FCLSH_HIP(hipGetLastError());
        p2k = keys;
        p2v = sv;
    }
    if (marks) FCLSH_HIP(hipEventRecord(marks[3], st));
    if (packed)
        return launch_pass2<uint16_t, true>(p2k, p2v, L, n, gstart, gbits2, lo_bits2, gk,
                                            static_cast<uint16_t *>(tkeys), tids, dir, rest, rest_count, tmpv, mode,
                                            p2_fallback, st, marks);
    if (table_key_bytes(dir_bits) == 2)
        return launch_pass2<uint16_t, false>(p2k, p2v, L, n, gstart, gbits2, lo_bits2, gk,
                                             static_cast<uint16_t *>(tkeys), tids, dir, rest, rest_count, tmpv, mode,
                                             p2_fallback, st, marks);
    return launch_pass2<uint32_t, false>(p2k, p2v, L, n, gstart, gbits2, lo_bits2, gk, static_cast<uint32_t *>(tkeys),
                                         tids, dir, rest, rest_count, tmpv, mode, p2_fallback, st, marks);
}

}  // namespace fclsh
