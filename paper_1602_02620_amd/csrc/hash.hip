// Alg. 2 of the paper on gfx950: all L integer bucket keys of a point in
// O(d + L log L).
//
//   sketch   t_j = sum of b_c over coordinates c of the part with x_c = 1
//            and m(c) = j (Alg. 2 lines 2-8; the specific construction is the
//            case of at most one coordinate per column, 0-padded)
//   FHT      F = H t with the Sylvester Hadamard matrix (Alg. 2 line 10)
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
//   * z = (S'' + 2^52) - F''_v holds 2y in the low 52 mantissa bits, so
//     lo32(z) >> 1 = y mod 2^31 and hi32(z) & 0xFFFFF = y >> 31; since
//     2^31 = 1 (mod P) the key is their sum, reduced by one conditional
//     subtraction of P.
//
// Layout.  A "unit" is one (point, part).  G lanes cooperate on a unit and
// each holds V = D/G sketch entries in registers: lane sub-index s owns
// columns j = s*V + k, k < V.  The in-register butterflies cover the low
// log2(V) index bits, lane exchanges the high log2(G) bits; afterwards lane s
// holds F_v for v = s*V + k (natural order).  Lanes are unit-fastest within a
// wave, so for each k the lanes of one sub-index write consecutive points of
// one table: keys are stored table-major [T][n], T = p*(D-1) + (v-1).
#include "common.h"

namespace fclsh {

namespace {

constexpr double kTwo52 = 4503599627370496.0;

template <int LOGD>
struct Shape {
    static constexpr int D = 1 << LOGD;
    static constexpr int G = D > 64 ? D / 64 : 1;  // lanes per unit
    static constexpr int V = D / G;                // sketch entries per lane
    static constexpr int U = 64 / G;               // units per wave
};

template <int LOGD>
__global__ __launch_bounds__(256) void fht_hash_kernel(
    const uint64_t *__restrict__ pts, int64_t m, int W, const int32_t *__restrict__ seg,
    const int32_t *__restrict__ ecoord, const double *__restrict__ eb, int E,
    uint32_t *__restrict__ keys, int64_t key_stride) {
    using S = Shape<LOGD>;
    constexpr int D = S::D, G = S::G, V = S::V, U = S::U;
    extern __shared__ uint32_t xs[];

    const int lane = threadIdx.x & 63;
    const int wave = threadIdx.x >> 6;
    const int wpb = blockDim.x >> 6;
    const int s = lane / U;  // sub-index of this lane within its unit
    const int u = lane % U;  // unit slot within the wave
    const int p = blockIdx.y;
    const int stride = 2 * W + 1;  // dwords per staged point (+1 zero dword)
    uint32_t *wx = xs + wave * U * stride;
    const int64_t base = (int64_t(blockIdx.x) * wpb + wave) * U;

    // Stage the wave's U points (coalesced uint64 loads) into LDS as dwords.
    for (int e = lane; e < U * W; e += 64) {
        const int uu = e / W, w = e - uu * W;
        const int64_t i = base + uu;
        const uint64_t v = (i < m) ? pts[i * W + w] : 0ull;
        wx[uu * stride + 2 * w] = uint32_t(v);
        wx[uu * stride + 2 * w + 1] = uint32_t(v >> 32);
    }
    if (lane < U) wx[lane * stride + 2 * W] = 0u;
    __builtin_amdgcn_s_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup");

    const uint32_t *myx = wx + u * stride;
    const int32_t *sg = seg + p * (V + 1);
    const int32_t *ec = ecoord + int64_t(p) * E * G + s;
    const double *ebp = eb + int64_t(p) * E * G + s;

    // Sketch (Alg. 2 lines 2-8).
    double t[V];
#pragma unroll
    for (int k = 0; k < V; ++k) {
        double acc = 0.0;
        const int e1 = sg[k + 1];
        for (int e = sg[k]; e < e1; ++e) {
            const int c = ec[e * G];
            const uint32_t word = myx[c >> 5];
            const double bv = ebp[e * G];
            acc += ((word >> (c & 31)) & 1u) ? bv : 0.0;
        }
        t[k] = acc;
    }

    // Fast Hadamard transform (Alg. 2 line 10), in-register stages.
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
    // Stages across the G lanes of a unit (lane distance U << g).
#pragma unroll
    for (int g = 1; g < G; g <<= 1) {
        const double sgn = (s & g) ? -1.0 : 1.0;
#pragma unroll
        for (int k = 0; k < V; ++k) {
            const double o = __shfl_xor(t[k], g * U, 64);
            t[k] = fma(sgn, t[k], o);
        }
    }

    // S'' = F''_0 lives in sub-index 0 (lane u) at k = 0.
    const double Sm = __shfl(t[0], u, 64) + kTwo52;
    const int64_t i = base + u;
    if (i < m) {
        uint32_t *out = keys + int64_t(p) * (D - 1) * key_stride + i;
#pragma unroll
        for (int k = 0; k < V; ++k) {
            const int v = s * V + k;
            if (v == 0) continue;  // all-zero codeword, removed by Alg. 2
            const double z = Sm - t[k];
            const uint64_t zb = __double_as_longlong(z);
            uint32_t y = (uint32_t(zb) >> 1) + (uint32_t(zb >> 32) & 0xFFFFFu);
            y = min(y, y - kPrime);
            out[int64_t(v - 1) * key_stride] = y;
        }
    }
}

template <int LOGD>
fclsh_status launch_t(const Index &ix, const uint64_t *pts, int64_t m, uint32_t *keys,
                      int64_t key_stride, hipStream_t st) {
    using S = Shape<LOGD>;
    const HashPlan &pl = ix.plan;
    const size_t per_wave = size_t(S::U) * (2 * pl.W + 1) * 4;
    int wpb = int(65536 / per_wave);
    if (wpb > 4) wpb = 4;
    if (wpb < 1) return fail(FCLSH_EUNSUPPORTED, "point too wide for the hash kernel");
    const int64_t per_block = int64_t(wpb) * S::U;
    const int64_t nblk = (m + per_block - 1) / per_block;
    if (nblk > 0x7FFFFFFF) return fail(FCLSH_EINVAL, "too many points for one launch");
    dim3 grid(unsigned(nblk), unsigned(pl.t));
    hipLaunchKernelGGL(fht_hash_kernel<LOGD>, grid, dim3(64 * wpb), per_wave * wpb, st, pts, m,
                       pl.W, pl.seg, pl.coord, pl.bval, pl.E, keys, key_stride);
    FCLSH_HIP(hipGetLastError());
    return FCLSH_OK;
}

}  // namespace

fclsh_status build_hash_plan(Index *ix) {
    const Params &p = ix->prm;
    HashPlan &pl = ix->plan;
    const int D = p.D();
    pl.logD = p.rp + 1;
    pl.G = D > 64 ? D / 64 : 1;
    pl.V = D / pl.G;
    pl.U = 64 / pl.G;
    pl.t = p.t;
    pl.W = ix->W;
    const int G = pl.G, V = pl.V;
    const int32_t zero_slot = 64 * ix->W;  // coordinate reading the staged zero dword

    // column -> coordinates of each part
    std::vector<std::vector<std::vector<int32_t>>> lists(p.t, std::vector<std::vector<int32_t>>(D));
    for (int c = 0; c < p.d; ++c) lists[p.part[c]][p.col[c]].push_back(c);

    std::vector<int32_t> seg(size_t(p.t) * (V + 1), 0);
    int E = 0;
    for (int q = 0; q < p.t; ++q) {
        int32_t *sq = &seg[size_t(q) * (V + 1)];
        for (int k = 0; k < V; ++k) {
            size_t mx = 0;
            for (int s = 0; s < G; ++s) mx = std::max(mx, lists[q][s * V + k].size());
            sq[k + 1] = sq[k] + int32_t(mx);
        }
        E = std::max(E, int(sq[V]));
    }
    pl.E = std::max(E, 1);
    std::vector<int32_t> coord(size_t(p.t) * pl.E * G, zero_slot);
    std::vector<double> bval(size_t(p.t) * pl.E * G, 0.0);
    for (int q = 0; q < p.t; ++q) {
        const int32_t *sq = &seg[size_t(q) * (V + 1)];
        for (int k = 0; k < V; ++k)
            for (int s = 0; s < G; ++s) {
                const auto &lst = lists[q][s * V + k];
                for (size_t a = 0; a < lst.size(); ++a) {
                    const size_t e = size_t(sq[k]) + a;
                    const size_t at = (size_t(q) * pl.E + e) * G + s;
                    const int c = lst[a];
                    coord[at] = c;
                    const uint64_t b = p.b[c];
                    bval[at] = double((b & 1) ? b + kPrime : b);
                }
            }
    }
    FCLSH_TRY(dev_alloc(ix, reinterpret_cast<void **>(&pl.seg), seg.size() * 4, "hash plan"));
    FCLSH_TRY(dev_alloc(ix, reinterpret_cast<void **>(&pl.coord), coord.size() * 4, "hash plan"));
    FCLSH_TRY(dev_alloc(ix, reinterpret_cast<void **>(&pl.bval), bval.size() * 8, "hash plan"));
    FCLSH_HIP(hipMemcpy(pl.seg, seg.data(), seg.size() * 4, hipMemcpyHostToDevice));
    FCLSH_HIP(hipMemcpy(pl.coord, coord.data(), coord.size() * 4, hipMemcpyHostToDevice));
    FCLSH_HIP(hipMemcpy(pl.bval, bval.data(), bval.size() * 8, hipMemcpyHostToDevice));
    return FCLSH_OK;
}

fclsh_status launch_hash(const Index &ix, const uint64_t *pts, int64_t m, uint32_t *keys,
                         int64_t key_stride, hipStream_t st) {
    if (m == 0) return FCLSH_OK;
    switch (ix.plan.logD) {
        case 1: return launch_t<1>(ix, pts, m, keys, key_stride, st);
        case 2: return launch_t<2>(ix, pts, m, keys, key_stride, st);
        case 3: return launch_t<3>(ix, pts, m, keys, key_stride, st);
        case 4: return launch_t<4>(ix, pts, m, keys, key_stride, st);
        case 5: return launch_t<5>(ix, pts, m, keys, key_stride, st);
        case 6: return launch_t<6>(ix, pts, m, keys, key_stride, st);
        case 7: return launch_t<7>(ix, pts, m, keys, key_stride, st);
        case 8: return launch_t<8>(ix, pts, m, keys, key_stride, st);
        case 9: return launch_t<9>(ix, pts, m, keys, key_stride, st);
        case 10: return launch_t<10>(ix, pts, m, keys, key_stride, st);
        case 11: return launch_t<11>(ix, pts, m, keys, key_stride, st);
        case 12: return launch_t<12>(ix, pts, m, keys, key_stride, st);
        default: return fail(FCLSH_EUNSUPPORTED, "Hadamard order 2^%d", ix.plan.logD);
    }
}

}  // namespace fclsh
