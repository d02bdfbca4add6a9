// Index parameters: Alg. 1 pre-processing (coordinate permutation and
// contiguous partitioning into t parts) and the random draws of Alg. 2 (per
// part a mapping into 2^(r'+1) Hadamard columns, Eq. (5), or a column
// permutation for the 0-padded specific construction; the seed vector b of
// Eq. (1)).  Host only.
#include <cstdarg>
#include <cstring>

#include "common.h"

namespace fclsh {

namespace {

thread_local std::string g_last_error;

// SplitMix64 (Steele, Lea & Flood, OOPSLA 2014) in counter form: draw number k
// of the stream seeded with s is the 64-bit finaliser applied to s + (k+1)*gamma.
class CounterRng {
   public:
    explicit CounterRng(uint64_t seed) : seed_(seed) {}
    uint64_t next() {
        ++count_;
        uint64_t x = seed_ + count_ * 0x9E3779B97F4A7C15ULL;
        x ^= x >> 30;
        x *= 0xBF58476D1CE4E5B9ULL;
        x ^= x >> 27;
        x *= 0x94D049BB133111EBULL;
        x ^= x >> 31;
        return x;
    }
    // Uniform in [0, bound): reject the lowest (2^64 mod bound) outputs.
    uint64_t below(uint64_t bound) {
        const uint64_t reject_under = (uint64_t(0) - bound) % bound;
        for (;;) {
            uint64_t x = next();
            if (x >= reject_under) return x % bound;
        }
    }
    // In-place uniform shuffle of v (swap v[i] with v[below(i+1)], i descending).
    void shuffle(std::vector<int32_t> &v) {
        for (size_t i = v.size(); i-- > 1;) {
            size_t j = size_t(below(uint64_t(i) + 1));
            std::swap(v[i], v[j]);
        }
    }

   private:
    uint64_t seed_;
    uint64_t count_ = 0;
};

}  // namespace

void set_error(const char *fmt, ...) {
    char buf[1024];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    g_last_error = buf;
}

fclsh_status fail(fclsh_status st, const char *fmt, ...) {
    char buf[1024];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    g_last_error = buf;
    return st;
}

const char *last_error_cstr() { return g_last_error.c_str(); }

fclsh_status check_params(const Params &p) {
    const int dmax = p.sparse ? kMaxSparseDims : kMaxDims;
    if (p.d <= 0 || p.d > dmax) return fail(FCLSH_EUNSUPPORTED, "d=%d outside [1, %d]", p.d, dmax);
    if (p.rep < 1 || (p.rep > 1 && p.t != 1))
        return fail(FCLSH_EINVAL, "replication (%d copies) needs a single part", p.rep);
    if (p.sparse && p.rep != 1) return fail(FCLSH_EUNSUPPORTED, "replication of sparse points");
    if (p.dd() > dmax)
        return fail(FCLSH_EUNSUPPORTED, "%d copies of d=%d exceed %d coordinates", p.rep, p.d, dmax);
    if (p.t < 1 || p.t > kMaxParts || p.t > p.d)
        return fail(FCLSH_EUNSUPPORTED, "t=%d parts unsupported for d=%d", p.t, p.d);
    if (p.rp < 0 || p.rp + 1 > kMaxLogD)
        return fail(FCLSH_EUNSUPPORTED, "per-part radius r'=%d: 2^(r'+1) exceeds %d columns", p.rp,
                    1 << kMaxLogD);
    // a replicated point has rep times the distance (Alg. 1)
    if (p.r < 0 || p.r * p.rep / p.t > p.rp)
        return fail(FCLSH_EINVAL, "radius r=%d not covered by t=%d parts of radius %d", p.r, p.t, p.rp);
    const int dd = p.dd();
    if ((int)p.part.size() != dd || (int)p.col.size() != dd || (int)p.b.size() != dd)
        return fail(FCLSH_EINVAL, "parameter arrays must have d * replicate entries");
    std::vector<int> seen(p.t, 0);
    for (int c = 0; c < dd; ++c) {
        if (p.part[c] < 0 || p.part[c] >= p.t) return fail(FCLSH_EINVAL, "part[%d]=%d out of range", c, p.part[c]);
        if (p.col[c] < 0 || p.col[c] >= p.D()) return fail(FCLSH_EINVAL, "col[%d]=%d out of range", c, p.col[c]);
        if (p.b[c] >= kPrime) return fail(FCLSH_EINVAL, "b[%d] not below the prime", c);
        seen[p.part[c]] = 1;
    }
    for (int q = 0; q < p.t; ++q)
        if (!seen[q]) return fail(FCLSH_EINVAL, "part %d has no coordinates", q);
    return FCLSH_OK;
}

fclsh_status derive_params(int d0, int r, uint64_t seed, const fclsh_build_opts *opts, Params *out, bool sparse) {
    if (d0 <= 0 || r < 0) return fail(FCLSH_EINVAL, "need d > 0 and r >= 0 (d=%d r=%d)", d0, r);
    const int dmax = sparse ? kMaxSparseDims : kMaxDims;
    if (d0 > dmax) return fail(FCLSH_EUNSUPPORTED, "d=%d exceeds %d", d0, dmax);
    if (opts && opts->replicate < 0) return fail(FCLSH_EINVAL, "negative replicate");
    if (opts && opts->prime != 0 && opts->prime != kPrime)
        return fail(FCLSH_EUNSUPPORTED, "only the prime 2^31-1 is supported");
    // Alg. 1, first branch: rep copies of every point, so a radius r becomes
    // rep * r on rep * d coordinates, with one part
    const int rep = (opts && opts->replicate > 1) ? opts->replicate : 1;
    if (rep > 1 && opts->partitions > 1)
        return fail(FCLSH_EINVAL, "replication and partitioning are exclusive (Alg. 1)");
    if (rep > 1 && sparse) return fail(FCLSH_EUNSUPPORTED, "replication of sparse points");
    if (int64_t(rep) * d0 > dmax)
        return fail(FCLSH_EUNSUPPORTED, "%d copies of d=%d exceed %d coordinates", rep, d0, dmax);
    const int d = rep * d0;  // coordinates the family is drawn for
    r *= rep;
    // Sec. 4.1 / Sec. 4.3: partition only for large radii (r >= 10, two parts).
    int t = rep > 1 ? 1 : (opts && opts->partitions > 0) ? opts->partitions : (r >= 10 ? 2 : 1);
    if (t > d || t > kMaxParts) return fail(FCLSH_EUNSUPPORTED, "t=%d parts for d=%d", t, d);
    int rp = r / t;  // pigeonhole: some part keeps at most floor(r/t) differences
    if (rp + 1 > kMaxLogD)
        return fail(FCLSH_EUNSUPPORTED, "per-part radius %d needs 2^%d columns (max %d)", rp, rp + 1,
                    1 << kMaxLogD);
    const int D = 1 << (rp + 1);
    // Sec. 3.3 variant: column 0 (the all-zero column of every codeword) is
    // never a target, so the columns drawn from are 1..D-1
    const bool skip0 = opts && opts->exclude_column0;
    const int ncols = skip0 ? D - 1 : D, col0 = skip0 ? 1 : 0;

    Params p;
    p.sparse = sparse;
    p.d = d0;
    p.r = r / rep;
    p.rep = rep;
    p.t = t;
    p.rp = rp;
    p.part.assign(d, 0);
    p.col.assign(d, 0);
    p.b.assign(d, 0);

    CounterRng rng(seed);
    std::vector<int32_t> order(d);
    for (int c = 0; c < d; ++c) order[c] = c;
    if (t > 1) rng.shuffle(order);  // Alg. 1: permute before partitioning

    const int block = d / t;
    std::vector<int32_t> cols(ncols);
    for (int q = 0; q < t; ++q) {
        const int begin = q * block;
        const int end = (q + 1 == t) ? d : begin + block;
        const int dq = end - begin;
        if (dq <= ncols) {
            // specific construction: random permutation of the allowed
            // columns, the part's coordinates take its first dq entries
            for (int j = 0; j < ncols; ++j) cols[j] = col0 + j;
            rng.shuffle(cols);
            for (int k = 0; k < dq; ++k) {
                p.part[order[begin + k]] = q;
                p.col[order[begin + k]] = cols[k];
            }
        } else {
            // general construction: i.i.d. uniform allowed column per coordinate
            for (int k = 0; k < dq; ++k) {
                p.part[order[begin + k]] = q;
                p.col[order[begin + k]] = col0 + int32_t(rng.below(uint64_t(ncols)));
            }
        }
    }
    for (int c = 0; c < d; ++c) p.b[c] = rng.below(kPrime);
    *out = std::move(p);
    return FCLSH_OK;
}

}  // namespace fclsh
