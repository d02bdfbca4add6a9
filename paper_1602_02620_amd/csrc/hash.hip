// Alg. 2 of the paper on gfx950: all L integer bucket keys of a point in
// O(d + L log L).
//
//   sketch   t_j = sum of b_c over coordinates c of the part with x_c = 1
//            and m(c) = j (the sketch of Alg. 2; the specific construction is the
//            case of at most one coordinate per column, 0-padded)
//   FHT      F = H t with the Sylvester Hadamard matrix (Alg. 2, Eq. (6))
//   keys     h_v = (S - F_v) / 2 mod P with S = sum_j t_j (= F_0), v >= 1
//            (Eq. (6); the v = 0 value is the all-zero codeword, dropped)
//
// Arithmetic.  The butterflies run in fp64, which is exact here: every
// sketch entry is an integer < 2^43 and |F_v| <= sum_j t_j < 2^43, far below
// 2^53.  fp64 adds are full rate on CDNA4, so a butterfly costs one VALU op
// per output.  Two exact rewrites remove the halving and the generic modulo:
//   * each b_c enters the sketch as its even representative b''_c in [0, 2P)
//     (b'' = b if b is even, else b + P), i.e. 2 * (b / 2 mod P); then
//     S'' - F''_v = 2 * y with y = (S - F_v)/2 (mod P) and y < 2^42;
//   * z = (S'' + 2^52) - F''_v = 2^52 + 2y exactly (the exponent word is
//     fixed), so lo32(z) >> 1 = y mod 2^31 and hi32(z) - hi32(2^52) = y >> 31;
//     since 2^31 = 1 (mod P) the key is their sum, reduced by one
//     conditional subtraction of P.
//
// Layout.  A "unit" is one (point, part).  G lanes cooperate on a unit and
// each holds V = D/G sketch entries in registers: lane sub-index s owns
// columns j = s*V + k, k < V.  The in-register butterflies cover the low
// log2(V) index bits, lane exchanges the high log2(G) bits; afterwards lane s
// holds F_v for v = s*V + k (natural order).  Lanes are unit-fastest within a
// wave, so for each k the lanes of one sub-index write consecutive points of
// one table: keys are stored table-major [T][n], T = p*(D-1) + (v-1).
//
// Points given by their nonzero coordinates take a second kernel that builds
// the sketch from the nonzeros alone (O(nnz + L log L) per point) and shares
// the FHT, key extraction and write-out.
#include <algorithm>

#include "common.h"

namespace fclsh {

namespace {

constexpr double kTwo52 = 4503599627370496.0;
constexpr uint32_t kHiWord52 = 0x43300000u;  // high word of 2^52 as a double

// A coordinate c as the gather table holds it: the byte offset of its dword
// in the staged point (4 * (c >> 5), below 2^16) in the high half, its bit
// (c & 31) in the low bits.  The dword's address is then one add with a
// word-select operand (SDWA), and the bit field extract reads the entry as
// its offset (the hardware uses its low 5 bits).
__host__ __device__ constexpr uint32_t coord_entry(uint32_t c) { return ((c >> 5) << 18) | (c & 31u); }

// All ones if the coordinate of entry e is set in the staged point x, else
// zero.
__device__ inline uint32_t coord_mask(const uint32_t *x, uint32_t e) {
    const uint32_t w = *reinterpret_cast<const uint32_t *>(reinterpret_cast<const char *>(x) + (e >> 16));
    return uint32_t(__builtin_amdgcn_sbfe(int32_t(w), e, 1u));
}

// Shape of one launch: V = 2^LOGV sketch entries per lane, G lanes per unit
// (point, part), U = 64/G units per wave.
template <int LOGD, int LOGV>
struct Shape {
    static constexpr int D = 1 << LOGD;
    static constexpr int V = 1 << LOGV;
    static constexpr int LOGG = LOGD - LOGV;
    static constexpr int G = 1 << LOGG;
    static constexpr int LOGU = 6 - LOGG;
    static constexpr int U = 1 << LOGU;
    static_assert(LOGG >= 0 && LOGG <= 6, "G must divide a wave");
    // Cross-lane stage b (lane bit LOGU + b, partner distance U << b) is a
    // "swap" stage when the distance is 32: a permlane swap of register
    // pairs (k, k ^ 2^q), q = LOGV - LOGG + b, moves index bit LOGV + b into
    // register bit q and the (already transformed) index bit q into the lane
    // bit; the butterfly then runs inside each lane.
    static constexpr bool swap_stage(int b) { return LOGU + b >= 5; }
    static constexpr int swap_reg(int b) { return LOGV - LOGG + b; }
    // Index bit held by register bit r after all stages.
    static constexpr int reg_bit_index(int r) {
        for (int b = 0; b < LOGG; ++b)
            if (swap_stage(b) && swap_reg(b) == r) return LOGV + b;
        return r;
    }
    // Index bits carried by register number k.
    static constexpr int vreg(int k) {
        int v = 0;
        for (int r = 0; r < LOGV; ++r)
            if ((k >> r) & 1) v |= 1 << reg_bit_index(r);
        return v;
    }
};

// The value of lane ^ DIST (DIST in 1, 2, 4, 8, 16): a ds_swizzle in bit
// mode (and-mask 0x1F, xor-mask DIST within each 32 lanes) per dword.  The
// swizzle runs in the LDS pipe, so these stages leave the VALU to the
// butterflies: a DPP move would take a VALU slot per dword, and a permlane16
// swap stage a VALU slot per dword plus an in-lane butterfly (hash on mid
// 0.644 -> 0.622 ms with distance 16 as a swizzle stage).
template <int DIST>
__device__ inline double xor_lane_f64(double x) {
    static_assert(DIST == 1 || DIST == 2 || DIST == 4 || DIST == 8 || DIST == 16, "swizzle distance");
    const uint64_t u = __double_as_longlong(x);
    const int lo = __builtin_amdgcn_ds_swizzle(int(uint32_t(u)), (DIST << 10) | 0x1F);
    const int hi = __builtin_amdgcn_ds_swizzle(int(uint32_t(u >> 32)), (DIST << 10) | 0x1F);
    return __longlong_as_double((int64_t(uint32_t(hi)) << 32) | uint32_t(lo));
}

// After the swap, a holds the partner-pair element with the partner-lane
// index bit 0 and b the one with it 1, in every lane (distance 32).
__device__ inline void swap32_f64(double &a, double &b) {
    const uint64_t ua = __double_as_longlong(a), ub = __double_as_longlong(b);
    uint32_t alo = uint32_t(ua), ahi = uint32_t(ua >> 32), blo = uint32_t(ub), bhi = uint32_t(ub >> 32);
    auto l = __builtin_amdgcn_permlane32_swap(alo, blo, false, false);
    auto h = __builtin_amdgcn_permlane32_swap(ahi, bhi, false, false);
    alo = l[0]; blo = l[1]; ahi = h[0]; bhi = h[1];
    a = __longlong_as_double((int64_t(ahi) << 32) | alo);
    b = __longlong_as_double((int64_t(bhi) << 32) | blo);
}

// Cross-lane stages B .. LOGG - 2 (distances U << B below 32, swizzles);
// the last one (distance 32, a swap stage) is fused with the key
// extraction's subtraction in fht_unit.
template <int LOGD, int LOGV, int B>
__device__ inline void cross_stages(double (&t)[1 << LOGV], int lane) {
    using S = Shape<LOGD, LOGV>;
    if constexpr (B < S::LOGG - 1) {
        constexpr int dist = S::U << B;
        static_assert(!S::swap_stage(B), "only the last cross-lane stage swaps");
        const double sgn = (lane & dist) ? -1.0 : 1.0;
#pragma unroll
        for (int k = 0; k < S::V; ++k) t[k] = fma(sgn, t[k], xor_lane_f64<dist>(t[k]));
        cross_stages<LOGD, LOGV, B + 1>(t, lane);
    }
}

// Waves per workgroup by Hadamard order, so that a workgroup's stage rows
// (NW*U points of one table) are at least 64 bytes, and 128 where LDS allows:
// measured on this GPU, writing 2 GB of such rows at a row stride of n keys
// runs at 1.3 TB/s with 16-byte rows, 3.8 TB/s with 64-byte rows and
// 5.5 TB/s with 128-byte or wider rows (a contiguous stream: 4.8 TB/s).
template <int LOGD, int LOGV>
constexpr int hash_waves() {
    return LOGV == 4 ? (LOGD == 8 ? 8 : 4) : LOGD == 9 || LOGD == 10 ? 8 : LOGD == 11 ? 16 : 4;
}

// Waves per workgroup of the sparse kernel (its accumulators, 8 bytes per
// column and point, take twice the stage's LDS).
template <int LOGD>
constexpr int sparse_waves() { return 4; }

// LDS staging of a block's keys: rows indexed by the Hadamard row v in
// [0, D) (row 0, the dropped all-zero codeword, is never written), each of
// PB = NW*U points, row v at v*PB + (v >> SH)*PAD.  (PAD, SH) per order from
// a model of the 64 LDS banks under which both access patterns are
// conflict-free: a wave's staging store (its G sub-lanes' rows, which differ
// in high index bits, times its U points) and a wave's write-out read (PB
// consecutive words of 64/PB consecutive rows).  Since SH <= log2(G), the
// padding term is additive over the disjoint index bits a lane and a
// register contribute (a lane's staging stores are one base plus
// constants), and over v = v0 + G*k with v0 < G (a thread's write-out reads
// are one base plus constants).
template <int LOGD>
constexpr int stage_pad() {
    return LOGD <= 5 ? 0 : LOGD == 6 ? 4 : LOGD <= 8 ? 8 : LOGD == 9 ? 4 : LOGD == 10 ? 2 : 1;
}
template <int LOGD>
constexpr int stage_shift() { return LOGD <= 5 ? 0 : LOGD == 6 ? 1 : LOGD == 7 ? 2 : LOGD <= 11 ? 3 : 4; }

template <int LOGD, int PB>
__device__ __host__ constexpr int stage_index(int v, int col) {
    return v * PB + (v >> stage_shift<LOGD>()) * stage_pad<LOGD>() + col;
}

template <int LOGD, int PB>
constexpr size_t stage_words() {
    return size_t(stage_index<LOGD, PB>((1 << LOGD) - 1, PB - 1)) + 1;
}

// Index bits of the output held by this lane (see Shape).
template <int LOGD, int LOGV>
__device__ inline int lane_rows(int lane) {
    using S = Shape<LOGD, LOGV>;
    int vlane = 0;
#pragma unroll
    for (int b = 0; b < S::LOGG; ++b)
        if ((lane >> (S::LOGU + b)) & 1) vlane |= 1 << (S::swap_stage(b) ? S::swap_reg(b) : LOGV + b);
    return vlane;
}

// The FHT of a unit's sketch (Alg. 2), then z_v = S'' + 2^52 - F''_v in
// place of each transform value F''_v (S'' = F''_0).  t holds the lane's V
// sketch entries.
template <int LOGD, int LOGV>
__device__ inline void fht_unit(double (&t)[1 << LOGV], int lane) {
    using S = Shape<LOGD, LOGV>;
    constexpr int V = S::V, U = S::U;
    // Fast Hadamard transform (Alg. 2): in-register stages ...
#pragma unroll
    for (int h = 1; h < V; h <<= 1) {
#pragma unroll
        for (int k = 0; k < V; ++k) {
            if (!(k & h)) {
                const double a = t[k], b = t[k | h];
                t[k] = a + b;
                t[k | h] = a - b;
            }
        }
    }
    // ... then the stages across the G lanes of a unit, nearest partners
    // first (the stages commute; this order keeps the register pressure of
    // the DPP stages away from the key extraction)
    cross_stages<LOGD, LOGV, 0>(t, lane);
    if constexpr (S::LOGG == 0) {
        const double Sm = t[0] + kTwo52;
#pragma unroll
        for (int k = 0; k < V; ++k) t[k] = Sm - t[k];
    } else {
        // the last stage (distance 32: LOGU + LOGG - 1 = 5), fused with the
        // subtraction: with c = Sm - a, the pair's z values are c - b and
        // c + b (integers below 2^53: exact).  F''_0 = a + b of register
        // pair 0 in the unit's lane with s = 0.
        static_assert(S::swap_stage(S::LOGG - 1), "the last cross-lane stage is a swap stage");
        constexpr int q = S::swap_reg(S::LOGG - 1);
        double a0 = t[0], b0 = t[1 << q];
        swap32_f64(a0, b0);
        const double Sm = __shfl(a0 + b0, lane & (U - 1), 64) + kTwo52;
#pragma unroll
        for (int k = 0; k < V; ++k) {
            if (!(k & (1 << q))) {
                double a = a0, b = b0;
                if (k != 0) {
                    a = t[k];
                    b = t[k | (1 << q)];
                    swap32_f64(a, b);
                }
                const double c = Sm - a;
                t[k] = c - b;
                t[k | (1 << q)] = c + b;
            }
        }
    }
}

// The unit's keys from z = S'' + 2^52 - F'': y[k] = h_v of the row held in
// register k (z = 2^52 + 2y exactly, 2y < 2^44: the high word is the
// exponent word kHiWord52 plus 2y >> 32, so y mod P (2^31 = 1) is
// (lo >> 1) + hi - kHiWord52, below 2P).
template <int LOGV>
__device__ inline void extract_keys(const double (&z)[1 << LOGV], uint32_t (&y)[1 << LOGV]) {
#pragma unroll
    for (int k = 0; k < (1 << LOGV); ++k) {
        const uint64_t zb = __double_as_longlong(z[k]);
        const uint32_t half = uint32_t(zb) >> 1, hi = uint32_t(zb >> 32);
        uint32_t y2;  // half + hi - kHiWord52, below 2P, in one three-operand add
        __asm__("v_add3_u32 %0, %1, %2, %3" : "=v"(y2) : "v"(half), "v"(hi), "s"(0u - kHiWord52));
        y[k] = min(y2, y2 - kPrime);
    }
}

// A unit's keys h_v, v >= 1, into the stage at column wave*U + u.
template <int LOGD, int LOGV, int NW>
__device__ inline void stage_keys(const uint32_t (&y)[1 << LOGV], int lane, int wave, uint32_t *stage) {
    using S = Shape<LOGD, LOGV>;
    constexpr int V = S::V, U = S::U, PB = NW * U;
    constexpr int PAD = stage_pad<LOGD>(), SH = stage_shift<LOGD>();
    static_assert(SH <= S::LOGG, "the stage padding must split over lane and register index bits");
    const int u = lane & (U - 1);
    const int vlane = lane_rows<LOGD, LOGV>(lane);
    // stage_index(vlane | vr, wave * U + u), split into a lane base and a
    // per-register constant
    const int sbase = vlane * PB + (vlane >> SH) * PAD + wave * U + u;
#pragma unroll
    for (int k = 0; k < V; ++k) {
        const int vr = S::vreg(k);
        if (vr == 0 && vlane == 0) continue;  // row 0: all-zero codeword, dropped
        stage[sbase + vr * PB + (vr >> SH) * PAD] = y[k];
    }
}

// The block's staged keys to the table-major key array: thread t writes
// column t % PB of rows v = t / PB + G k (the 64 NW threads cover G rows at
// a time), stage row v going to table p (D-1) + v - 1, for the PB points
// from first_point on.  Rows of at least 64 bytes are written with
// non-temporal stores (the kernel never reads them back); shorter rows keep
// the normal path, whose L2 merges the neighbouring workgroups' pieces of a
// line.
template <int LOGD, int LOGV, int NW>
__device__ inline void write_stage(const uint32_t *stage, uint32_t *__restrict__ keys, int64_t key_stride, int p,
                                   int64_t first_point, int64_t m) {
    using S = Shape<LOGD, LOGV>;
    constexpr int G = S::G, U = S::U, D = S::D, PB = NW * U;
    constexpr int PAD = stage_pad<LOGD>(), SH = stage_shift<LOGD>();
    const int v0 = threadIdx.x / PB;
    const int col = threadIdx.x % PB;
    const int64_t i = first_point + col;
    if (i >= m) return;
    const uint32_t *src = stage + stage_index<LOGD, PB>(v0, col);
    uint32_t *row1 = keys + (int64_t(p) * (D - 1) + v0) * key_stride + i;  // table of v = v0 + 1
    constexpr int NK = D / G;
    constexpr int CH = NK < 16 ? NK : 16;
    constexpr int KSTEP = G * PB + (G >> SH) * PAD;  // stage_index(v + G, c) - stage_index(v, c)
#pragma unroll
    for (int k0 = 0; k0 < NK; k0 += CH) {
        uint32_t val[CH];
#pragma unroll
        for (int c = 0; c < CH; ++c) val[c] = src[(k0 + c) * KSTEP];
#pragma unroll
        for (int c = 0; c < CH; ++c) {
            const int k = k0 + c;
            if (k == 0 && v0 == 0) continue;  // v = 0: the dropped row
            uint32_t *dst = row1 + (int64_t(k) * G - 1) * key_stride;
            if constexpr (PB * 4 >= 64)
                __builtin_nontemporal_store(val[c], dst);
            else
                *dst = val[c];
        }
    }
}

// One workgroup of NW waves per (part, `rounds` x NW consecutive point
// groups), in XCD-contiguous order; in each round every wave takes one group
// of U consecutive points and the block writes the keys of its NW*U points
// out together.  Short-lived waves keep every SIMD full: a grid-stride loop over
// groups measured 1.9x slower on the mid workload, and the 512-column kernel
// runs one round (see hash_rounds).  The part's gather table (per in-lane
// column k and sub-lane s, the coordinate feeding it and its even
// representative b'') is staged in LDS once per workgroup.
template <int LOGD, int LOGV, bool SPECIFIC, int NW>
__global__ __launch_bounds__(64 * NW) void fht_hash_kernel(const uint64_t *__restrict__ pts, int64_t m, int W,
                                                       const int32_t *__restrict__ seg,
                                                       const uint2 *__restrict__ gtab, int E,
                                                       uint32_t *__restrict__ keys, int64_t key_stride,
                                                       int64_t nblk, int64_t nitems, int rounds) {
    using S = Shape<LOGD, LOGV>;
    constexpr int V = S::V, G = S::G, U = S::U;
    extern __shared__ __align__(16) uint32_t lds[];
    const int lane = threadIdx.x & 63;
    const int wave = threadIdx.x >> 6;
    const int s = lane >> S::LOGU;
    const int u = lane & (U - 1);
    // work item: (part p, `rounds` consecutive blocks of NW point groups),
    // XCD-contiguous
    const int64_t witem = xcd_contiguous_item(blockIdx.x, gridDim.x);
    if (witem >= nitems) return;  // grid padding
    const int p = int(witem / nblk);
    const int64_t c0 = (witem % nblk) * NW * rounds;  // the item's first point group
    const int stride = 2 * W + 1;
    uint2 *tab = reinterpret_cast<uint2 *>(lds);
    uint32_t *wx = lds + 2 * E * G + wave * U * stride;

    for (int i = threadIdx.x; i < E * G; i += 64 * NW) tab[i] = gtab[int64_t(p) * E * G + i];
    __syncthreads();

    // The block's keys are staged in LDS as rows of NW*U points, then written
    // out row by row: NW*U consecutive points of a table per row segment
    // instead of the U of one wave.
    uint32_t *stage = lds + 2 * E * G + NW * U * stride;
    const int64_t ngroups = (m + U - 1) / U;
    for (int64_t g0 = c0; g0 < c0 + NW * rounds && g0 < ngroups; g0 += NW) {  // workgroup-uniform
        const int64_t grp = g0 + wave;
        const int64_t base = grp * U;
        if (grp < ngroups) {  // wave-uniform
            for (int e = lane; e < U * W; e += 64) {
                const int uu = e / W, w = e - uu * W;
                const int64_t i = base + uu;
                const uint64_t v = (i < m) ? pts[i * W + w] : 0ull;
                wx[uu * stride + 2 * w] = uint32_t(v);
                wx[uu * stride + 2 * w + 1] = uint32_t(v >> 32);
            }
            if (lane < U) wx[lane * stride + 2 * W] = 0u;
            __asm__ volatile("" ::: "memory");
            __builtin_amdgcn_wave_barrier();
            const uint32_t *myx = wx + u * stride;

            // Sketch (Alg. 2)
            double t[V];
            if constexpr (SPECIFIC) {
#pragma unroll
                for (int k = 0; k < V; ++k) {
                    const uint2 en = tab[k * G + s];
                    t[k] = double(en.x & coord_mask(myx, en.y));
                }
            } else {
                // integer sums (at most d terms below 2^32: exact in 64
                // bits), one conversion per column
                const int32_t *sg = seg + p * (V + 1);
#pragma unroll
                for (int k = 0; k < V; ++k) {
                    uint64_t acc = 0;
                    const int e1 = sg[k + 1];
                    int e = sg[k];
                    // four entries at a time: their table reads, then their
                    // point reads, are in flight together (one at a time, an
                    // entry took two dependent LDS round trips; batched hash
                    // 1.83 -> 1.76 ms)
                    for (; e + 4 <= e1; e += 4) {
                        const uint2 a0 = tab[e * G + s], a1 = tab[(e + 1) * G + s];
                        const uint2 a2 = tab[(e + 2) * G + s], a3 = tab[(e + 3) * G + s];
                        const uint32_t m0 = coord_mask(myx, a0.y), m1 = coord_mask(myx, a1.y);
                        const uint32_t m2 = coord_mask(myx, a2.y), m3 = coord_mask(myx, a3.y);
                        acc += uint64_t(a0.x & m0) + uint64_t(a1.x & m1) + uint64_t(a2.x & m2) + uint64_t(a3.x & m3);
                    }
                    for (; e < e1; ++e) {
                        const uint2 en = tab[e * G + s];
                        acc += en.x & coord_mask(myx, en.y);
                    }
                    t[k] = double(acc);
                }
            }
            __asm__ volatile("" ::: "memory");
            __builtin_amdgcn_wave_barrier();
            uint32_t y[V];
            fht_unit<LOGD, LOGV>(t, lane);
            extract_keys<LOGV>(t, y);
            stage_keys<LOGD, LOGV, NW>(y, lane, wave, stage);
        }
        __syncthreads();
        write_stage<LOGD, LOGV, NW>(stage, keys, key_stride, p, g0 * U, m);
        __syncthreads();
    }
}

// The same keys for points given by their nonzero coordinates (CSR rows),
// in O(nnz + L log L) per point (the sparse case of Sec. 3.2).  Each wave
// accumulates its U points' sketches in LDS: the U rows are consecutive, so
// their nonzeros form one range, which the lanes stride over four loads at a
// time (a lane's row index only moves forward); every nonzero coordinate of
// the workgroup's part adds its even representative to its column with a
// 64-bit LDS atomic (two nonzeros may share a column).  The wave then reads
// its sketches into registers, and the FHT, key extraction, staging and
// write-out are the dense kernel's; the stage reuses the accumulators' LDS
// once every wave has read its sketches.  coord[c] = (even representative
// b''_c, part(c) << 16 | column(c)).  Row bounds are clamped to [0, nnz]
// and made non-decreasing, and columns outside [0, d) are skipped.
template <int LOGD, int LOGV, int NW>
__global__ __launch_bounds__(64 * NW) void fht_hash_sparse_kernel(
    const int64_t *__restrict__ ptr, const int32_t *__restrict__ cols, int64_t nnz, int d, int64_t m,
    const uint2 *__restrict__ coord, uint32_t *__restrict__ keys, int64_t key_stride, int64_t nblk,
    int64_t nitems) {
    using S = Shape<LOGD, LOGV>;
    constexpr int V = S::V, U = S::U, D = S::D;
    extern __shared__ __align__(16) uint64_t lds64[];
    const int lane = threadIdx.x & 63;
    const int wave = threadIdx.x >> 6;
    const int s = lane >> S::LOGU;
    const int u = lane & (U - 1);
    const int64_t witem = xcd_contiguous_item(blockIdx.x, gridDim.x);
    if (witem >= nitems) return;  // grid padding
    const int p = int(witem / nblk);
    const int64_t g0 = (witem % nblk) * NW;  // the workgroup's first point group
    const int64_t grp = g0 + wave;
    const int64_t ngroups = (m + U - 1) / U;
    double t[V];
    if (grp < ngroups) {  // wave-uniform
        uint64_t *acc = lds64 + int64_t(wave) * U * D;
        int64_t *starts = reinterpret_cast<int64_t *>(lds64 + NW * U * D) + wave * (U + 1);
        const int64_t r0 = grp * U;
        const int rows = int(min(int64_t(U), m - r0));
        // row starts: clamped, then a running maximum across the lanes
        long long v = lane <= rows ? (long long)min(max(ptr[r0 + lane], int64_t(0)), nnz) : 0ll;
#pragma unroll
        for (int o = 1; o < 64; o <<= 1) {
            const long long y = __shfl_up(v, o, 64);
            if (lane >= o) v = max(v, y);
        }
        if (lane <= rows) starts[lane] = v;
        if (rows == 64 && lane == 63) starts[64] = max(v, (long long)min(max(ptr[r0 + 64], int64_t(0)), nnz));
        for (int i = lane; i < U * D; i += 64) acc[i] = 0ull;
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
        __builtin_amdgcn_wave_barrier();
        const int64_t E0 = starts[0], E1 = starts[rows];
        int row = 0;  // the lane's current row: starts[row] <= e < starts[row + 1]
        constexpr int R = 4;
        for (int64_t e0 = E0 + lane; e0 < E1; e0 += 64 * R) {
            int32_t c[R];
#pragma unroll
            for (int k = 0; k < R; ++k) {
                const int64_t e = e0 + 64 * k;
                c[k] = e < E1 ? cols[e] : -1;
            }
            uint2 cw[R];
#pragma unroll
            for (int k = 0; k < R; ++k) cw[k] = uint32_t(c[k]) < uint32_t(d) ? coord[c[k]] : make_uint2(0u, ~0u);
#pragma unroll
            for (int k = 0; k < R; ++k) {
                const int64_t e = e0 + 64 * k;
                if (e >= E1) break;
                while (e >= starts[row + 1]) ++row;
                if (int(cw[k].y >> 16) == p)
                    __hip_atomic_fetch_add(&acc[row * D + int(cw[k].y & 0xFFFFu)], uint64_t(cw[k].x),
                                           __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WAVEFRONT);
            }
        }
        __builtin_amdgcn_fence(__ATOMIC_ACQ_REL, "wavefront");
        __builtin_amdgcn_wave_barrier();
        const uint64_t *mine = acc + u * D + s * V;
#pragma unroll
        for (int k = 0; k < V; ++k) t[k] = double(mine[k]);
    }
    __syncthreads();  // every wave has its sketch: the stage may overwrite the accumulators
    uint32_t *stage = reinterpret_cast<uint32_t *>(lds64);
    if (grp < ngroups) {
        uint32_t y[V];
        fht_unit<LOGD, LOGV>(t, lane);
        extract_keys<LOGV>(t, y);
        stage_keys<LOGD, LOGV, NW>(y, lane, wave, stage);
    }
    __syncthreads();
    write_stage<LOGD, LOGV, NW>(stage, keys, key_stride, p, g0 * U, m);
}

// Rounds of NW point groups per workgroup (the gather table is staged once
// for all of them), by measurement: short-lived workgroups (D' below 512)
// gain from several rounds, the 512-column kernel loses (hash times in ms
// for 1 / 2 / 4 / 8 rounds: D' = 512, 1M points: 0.68 / 0.79 / 0.75 / 0.76;
// D' = 128, 10M points: 1.45 / 1.36 / 1.33 / 1.31; D' = 128 with several
// coordinates per column, 4M points: 2.55 / 2.46 / 2.56 / 2.57).
inline int hash_rounds(int logD, bool specific) { return logD >= 9 ? 1 : specific ? 4 : 2; }

template <int LOGD, int LOGV>
fclsh_status launch_t(const Index &ix, const uint64_t *pts, int64_t m, uint32_t *keys, int64_t key_stride,
                      hipStream_t st) {
    using S = Shape<LOGD, LOGV>;
    constexpr int NW = hash_waves<LOGD, LOGV>();
    const HashPlan &pl = ix.plan;
    const size_t lds = size_t(pl.E) * S::G * 8 + size_t(NW) * S::U * (2 * pl.W + 1) * 4 +
                       stage_words<LOGD, NW * S::U>() * 4;
    if (lds > 160 * 1024) return fail(FCLSH_EUNSUPPORTED, "hash kernel LDS need %zu bytes", lds);
    const int64_t ngroups = (m + S::U - 1) / S::U;
    const int rounds = hash_rounds(LOGD, pl.specific);
    const int64_t nblk = (ngroups + NW * rounds - 1) / (NW * rounds);  // work items per part
    const int64_t nitems = nblk * pl.t;
    const int64_t grid = xcd_grid(nitems);
    if (grid > 0x7FFFFFFF) return fail(FCLSH_EUNSUPPORTED, "%lld points need too many workgroups", (long long)m);
    if (pl.specific)
        hipLaunchKernelGGL((fht_hash_kernel<LOGD, LOGV, true, NW>), dim3(unsigned(grid)), dim3(64 * NW), lds, st,
                           pts, m, pl.W, pl.seg, pl.gtab, pl.E, keys, key_stride, nblk, nitems, rounds);
    else
        hipLaunchKernelGGL((fht_hash_kernel<LOGD, LOGV, false, NW>), dim3(unsigned(grid)), dim3(64 * NW), lds, st,
                           pts, m, pl.W, pl.seg, pl.gtab, pl.E, keys, key_stride, nblk, nitems, rounds);
    FCLSH_HIP(hipGetLastError());
    return FCLSH_OK;
}

template <int LOGD, int LOGV>
fclsh_status launch_sparse_t(const Index &ix, const CsrRows &rows, int64_t m, uint32_t *keys, int64_t key_stride,
                             hipStream_t st) {
    using S = Shape<LOGD, LOGV>;
    constexpr int NW = sparse_waves<LOGD>();
    const HashPlan &pl = ix.plan;
    const size_t acc = size_t(NW) * S::U * S::D * 8 + size_t(NW) * (S::U + 1) * 8;  // sketches + row starts
    const size_t stage = stage_words<LOGD, NW * S::U>() * 4;
    const size_t lds = std::max(acc, stage);
    if (lds > 160 * 1024) return fail(FCLSH_EUNSUPPORTED, "sparse hash kernel LDS need %zu bytes", lds);
    const int64_t ngroups = (m + S::U - 1) / S::U;
    const int64_t nblk = (ngroups + NW - 1) / NW;  // work items per part
    const int64_t nitems = nblk * pl.t;
    const int64_t grid = xcd_grid(nitems);
    if (grid > 0x7FFFFFFF) return fail(FCLSH_EUNSUPPORTED, "%lld points need too many workgroups", (long long)m);
    hipLaunchKernelGGL((fht_hash_sparse_kernel<LOGD, LOGV, NW>), dim3(unsigned(grid)), dim3(64 * NW), lds, st,
                       rows.ptr, rows.cols, rows.nnz, ix.prm.d, m, pl.coord, keys, key_stride, nblk, nitems);
    FCLSH_HIP(hipGetLastError());
    return FCLSH_OK;
}

}  // namespace

// 32 sketch entries per lane (64 VGPRs of fp64), 64 only where a unit would
// otherwise need more than a wave (D = 4096).  The general construction at
// D = 64..256 takes 16 per lane: its gather loop keeps many loads in flight,
// and with half the registers for the sketch more waves fit a SIMD (4M
// points, D = 128: 2.24 -> 1.78 ms), while the specific construction lost
// with 16 (D = 512: 0.64 -> 0.87 ms).
int hash_log_v(int logD, bool specific) {
    if (!specific && logD >= 6 && logD <= 8) return 4;
    return logD <= 5 ? logD : (logD - 6 > 5 ? logD - 6 : 5);
}

fclsh_status build_hash_plan(Index *ix) {
    const Params &p = ix->prm;
    HashPlan &pl = ix->plan;
    const int D = p.D();
    pl.logD = p.rp + 1;
    pl.t = p.t;
    pl.W = ix->W;
    // column -> coordinates of each part
    std::vector<std::vector<std::vector<int32_t>>> lists(p.sparse ? 0 : p.t, std::vector<std::vector<int32_t>>(D));
    // (with replication, coordinate c of the replicated point is bit c mod d
    // of the point: each bit feeds one column per copy)
    size_t most = 0;
    if (!p.sparse) {
        for (int c = 0; c < p.dd(); ++c) lists[p.part[c]][p.col[c]].push_back(c);
        for (auto &lp : lists)
            for (auto &l : lp) most = std::max(most, l.size());
    }
    pl.specific = most <= 1;
    pl.logV = hash_log_v(pl.logD, pl.specific);
    pl.V = 1 << pl.logV;
    pl.G = D / pl.V;
    pl.U = 64 / pl.G;
    if (p.sparse) {
        // one (even representative, part << 16 | column) word pair per coordinate
        std::vector<uint32_t> coord(size_t(p.d) * 2);
        for (int c = 0; c < p.d; ++c) {
            const uint64_t b = p.b[c];
            coord[size_t(c) * 2] = uint32_t((b & 1) ? b + kPrime : b);
            coord[size_t(c) * 2 + 1] = uint32_t(p.part[c]) << 16 | uint32_t(p.col[c]);
        }
        FCLSH_TRY(dev_alloc(ix, reinterpret_cast<void **>(&pl.coord), coord.size() * 4, "hash plan"));
        FCLSH_HIP(hipMemcpy(pl.coord, coord.data(), coord.size() * 4, hipMemcpyHostToDevice));
        return FCLSH_OK;
    }
    const int G = pl.G, V = pl.V;
    const uint32_t zero_slot = coord_entry(uint32_t(64 * ix->W));  // reads the staged zero dword

    // in-lane column k of sub-lane s is Hadamard column s*V + k; entries of k
    // are padded to the longest list among the G sub-lanes
    std::vector<int32_t> seg(size_t(p.t) * (V + 1), 0);
    int E = 0;
    for (int q = 0; q < p.t; ++q) {
        int32_t *sq = &seg[size_t(q) * (V + 1)];
        for (int k = 0; k < V; ++k) {
            size_t mx = pl.specific ? 1 : 0;
            for (int s = 0; s < G; ++s) mx = std::max(mx, lists[q][s * V + k].size());
            sq[k + 1] = sq[k] + int32_t(mx);
        }
        E = std::max(E, int(sq[V]));
    }
    pl.E = std::max(E, 1);
    std::vector<uint32_t> tab(size_t(p.t) * pl.E * G * 2, 0);
    for (size_t i = 0; i < tab.size(); i += 2) tab[i + 1] = zero_slot;
    for (int q = 0; q < p.t; ++q) {
        const int32_t *sq = &seg[size_t(q) * (V + 1)];
        for (int k = 0; k < V; ++k)
            for (int s = 0; s < G; ++s) {
                const auto &lst = lists[q][s * V + k];
                for (size_t a = 0; a < lst.size(); ++a) {
                    const size_t at = ((size_t(q) * pl.E + size_t(sq[k]) + a) * G + s) * 2;
                    const int c = lst[a];
                    const uint64_t b = p.b[c];
                    tab[at] = uint32_t((b & 1) ? b + kPrime : b);  // even representative, < 2^32
                    tab[at + 1] = coord_entry(uint32_t(c % p.d));
                }
            }
    }
    FCLSH_TRY(dev_alloc(ix, reinterpret_cast<void **>(&pl.seg), seg.size() * 4, "hash plan"));
    FCLSH_TRY(dev_alloc(ix, reinterpret_cast<void **>(&pl.gtab), tab.size() * 4, "hash plan"));
    FCLSH_HIP(hipMemcpy(pl.seg, seg.data(), seg.size() * 4, hipMemcpyHostToDevice));
    FCLSH_HIP(hipMemcpy(pl.gtab, tab.data(), tab.size() * 4, hipMemcpyHostToDevice));
    return FCLSH_OK;
}

fclsh_status launch_hash(const Index &ix, const uint64_t *pts, int64_t m, uint32_t *keys,
                         int64_t key_stride, hipStream_t st) {
    if (m == 0) return FCLSH_OK;
    if (ix.plan.logV == 4 && ix.plan.logD >= 6) {
        switch (ix.plan.logD) {
            case 6: return launch_t<6, 4>(ix, pts, m, keys, key_stride, st);
            case 7: return launch_t<7, 4>(ix, pts, m, keys, key_stride, st);
            case 8: return launch_t<8, 4>(ix, pts, m, keys, key_stride, st);
            default: return fail(FCLSH_EUNSUPPORTED, "Hadamard order 2^%d with 16 entries per lane", ix.plan.logD);
        }
    }
    switch (ix.plan.logD) {
        case 1: return launch_t<1, 1>(ix, pts, m, keys, key_stride, st);
        case 2: return launch_t<2, 2>(ix, pts, m, keys, key_stride, st);
        case 3: return launch_t<3, 3>(ix, pts, m, keys, key_stride, st);
        case 4: return launch_t<4, 4>(ix, pts, m, keys, key_stride, st);
        case 5: return launch_t<5, 5>(ix, pts, m, keys, key_stride, st);
        case 6: return launch_t<6, 5>(ix, pts, m, keys, key_stride, st);
        case 7: return launch_t<7, 5>(ix, pts, m, keys, key_stride, st);
        case 8: return launch_t<8, 5>(ix, pts, m, keys, key_stride, st);
        case 9: return launch_t<9, 5>(ix, pts, m, keys, key_stride, st);
        case 10: return launch_t<10, 5>(ix, pts, m, keys, key_stride, st);
        case 11: return launch_t<11, 5>(ix, pts, m, keys, key_stride, st);
        case 12: return launch_t<12, 6>(ix, pts, m, keys, key_stride, st);
        default: return fail(FCLSH_EUNSUPPORTED, "Hadamard order 2^%d", ix.plan.logD);
    }
}

fclsh_status launch_hash_sparse(const Index &ix, const CsrRows &rows, int64_t m, uint32_t *keys, int64_t key_stride,
                                hipStream_t st) {
    if (m == 0) return FCLSH_OK;
    if (!ix.plan.coord) return fail(FCLSH_EINVAL, "the index holds dense points");
    switch (ix.plan.logD) {
        case 1: return launch_sparse_t<1, 1>(ix, rows, m, keys, key_stride, st);
        case 2: return launch_sparse_t<2, 2>(ix, rows, m, keys, key_stride, st);
        case 3: return launch_sparse_t<3, 3>(ix, rows, m, keys, key_stride, st);
        case 4: return launch_sparse_t<4, 4>(ix, rows, m, keys, key_stride, st);
        case 5: return launch_sparse_t<5, 5>(ix, rows, m, keys, key_stride, st);
        case 6: return launch_sparse_t<6, 5>(ix, rows, m, keys, key_stride, st);
        case 7: return launch_sparse_t<7, 5>(ix, rows, m, keys, key_stride, st);
        case 8: return launch_sparse_t<8, 5>(ix, rows, m, keys, key_stride, st);
        case 9: return launch_sparse_t<9, 5>(ix, rows, m, keys, key_stride, st);
        case 10: return launch_sparse_t<10, 5>(ix, rows, m, keys, key_stride, st);
        case 11: return launch_sparse_t<11, 5>(ix, rows, m, keys, key_stride, st);
        case 12: return launch_sparse_t<12, 6>(ix, rows, m, keys, key_stride, st);
        default: return fail(FCLSH_EUNSUPPORTED, "Hadamard order 2^%d", ix.plan.logD);
    }
}

}  // namespace fclsh
