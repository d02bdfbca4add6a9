// Host-side checks of the library, built with AddressSanitizer and
// UndefinedBehaviorSanitizer on the host code (the device code is compiled
// as usual) and run on a machine without a GPU.  It drives every host path
// that needs no device: parameter derivation and validation (dense and
// sparse sizes, replication, the column-0-excluded map, malformed arrays),
// Alg. 1's choice, the options struct, the layout of a query workspace in
// one buffer, the table-build sizing, and the argument checks of the entry
// points.  A sanitizer report aborts the run; a failed check prints it and
// exits with status 1.
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <limits>
#include <vector>

#include "../../paper_1602_02620_amd/csrc/common.h"

using namespace fclsh;

static int g_fail = 0;
#define CHECK(cond)                                                           \
    do {                                                                      \
        if (!(cond)) {                                                        \
            std::printf("check failed at line %d: %s\n", __LINE__, #cond);   \
            ++g_fail;                                                         \
        }                                                                     \
    } while (0)

static void params_grid() {
    const int ds[] = {1, 2, 5, 63, 64, 65, 100, 512, 1000, 4096};
    for (int d : ds)
        for (int r = 0; r <= 30; r += (r < 6 ? 1 : 5))
            for (int t : {0, 1, 2, 3, 64})
                for (int skip0 : {0, 1}) {
                    fclsh_build_opts o{};
                    o.struct_size = sizeof o;
                    o.partitions = t;
                    o.exclude_column0 = skip0;
                    Params p;
                    if (derive_params(d, r, 0x1234u + unsigned(d) * 7u + unsigned(r), &o, &p) != FCLSH_OK) continue;
                    CHECK(check_params(p) == FCLSH_OK);
                    CHECK(int(p.part.size()) == d && p.L() == p.t * (p.D() - 1));
                }
    for (int rep : {2, 3, 4, 8})
        for (int d : {1, 16, 100, 512, 1024, 2048})
            for (int r = 1; r <= 5; ++r) {
                fclsh_build_opts o{};
                o.struct_size = sizeof o;
                o.replicate = rep;
                Params p;
                if (derive_params(d, r, 99, &o, &p) != FCLSH_OK) continue;
                CHECK(check_params(p) == FCLSH_OK && p.dd() == rep * d && int(p.b.size()) == rep * d);
            }
    // sparse sizes
    for (int d : {4097, 28102, 140214, kMaxSparseDims})
        for (int r : {2, 7, 13, 29}) {
            Params p;
            fclsh_build_opts o{};
            o.struct_size = sizeof o;
            o.partitions = r >= 20 ? 3 : 0;
            CHECK(derive_params(d, r, 7, &o, &p, true) == FCLSH_OK);
            CHECK(p.sparse && check_params(p) == FCLSH_OK);
            Params q;
            CHECK(derive_params(d, r, 7, &o, &q, false) == FCLSH_EUNSUPPORTED);  // dense points stop at 4096
        }
    Params p;
    CHECK(derive_params(kMaxSparseDims + 1, 3, 1, nullptr, &p, true) == FCLSH_EUNSUPPORTED);
    CHECK(derive_params(0, 3, 1, nullptr, &p) == FCLSH_EINVAL);
    CHECK(derive_params(10, -1, 1, nullptr, &p) == FCLSH_EINVAL);
}

static void malformed_params() {
    Params base;
    CHECK(derive_params(40, 10, 5, nullptr, &base) == FCLSH_OK);
    {
        Params p = base;
        p.part[3] = p.t;  // part out of range
        CHECK(check_params(p) == FCLSH_EINVAL);
    }
    {
        Params p = base;
        p.col[0] = p.D();
        CHECK(check_params(p) == FCLSH_EINVAL);
    }
    {
        Params p = base;
        p.b[1] = kPrime;
        CHECK(check_params(p) == FCLSH_EINVAL);
    }
    {
        Params p = base;
        for (auto &x : p.part) x = 0;  // part 1 left empty
        CHECK(check_params(p) == FCLSH_EINVAL);
    }
    {
        Params p = base;
        p.col.pop_back();  // arrays of the wrong length
        CHECK(check_params(p) == FCLSH_EINVAL);
    }
    {
        Params p = base;
        p.r = p.t * (p.rp + 1);  // radius not covered by the parts
        CHECK(check_params(p) == FCLSH_EINVAL);
    }
}

static void entry_point_arguments() {
    int32_t rep = 0, parts = 0;
    CHECK(fclsh_preprocessing(1 << 20, 3, 2.0, &rep, &parts) == FCLSH_OK && rep == 3 && parts == 1);
    CHECK(fclsh_preprocessing(1 << 20, 40, 2.0, &rep, &parts) == FCLSH_OK && rep == 1 && parts == 4);
    CHECK(fclsh_preprocessing(int64_t(1) << 62, 1, 1.0000001, &rep, &parts) == FCLSH_OK && rep == 61);
    CHECK(fclsh_preprocessing(2, 1 << 30, 1e300, &rep, &parts) == FCLSH_OK && parts == (1 << 30));
    CHECK(fclsh_preprocessing(1 << 20, 3, std::nan(""), &rep, &parts) == FCLSH_EINVAL);
    CHECK(fclsh_preprocessing(1, 3, 2.0, &rep, &parts) == FCLSH_EINVAL);
    CHECK(fclsh_preprocessing(100, 3, 2.0, nullptr, &parts) == FCLSH_EINVAL);

    std::vector<int32_t> part(300), col(300);
    std::vector<uint64_t> b(300);
    int32_t t = 0, rp = 0;
    // the options struct read up to its struct_size
    struct {
        fclsh_build_opts o;
        char tail[16];
    } big{};
    for (uint32_t sz = 0; sz <= sizeof(fclsh_build_opts) + 8; sz += 4) {
        fclsh_build_opts o{};
        std::memset(&o, 0, sizeof o);
        o.struct_size = sz;
        o.partitions = 2;
        const fclsh_status s = fclsh_derive_params(300, 12, 5, &o, &t, &rp, part.data(), col.data(), b.data());
        if (sz < 4 || sz > sizeof(fclsh_build_opts))
            CHECK(s == FCLSH_EINVAL);
        else
            CHECK(s == FCLSH_OK && t == (sz >= 8 ? 2 : 2));  // r >= 10: two parts either way
    }
    big.o.struct_size = sizeof(fclsh_build_opts);
    big.o.test_flags = 2;  // unknown test flag bit
    CHECK(fclsh_derive_params(300, 12, 5, &big.o, &t, &rp, part.data(), col.data(), b.data()) == FCLSH_EINVAL);
    CHECK(fclsh_derive_params(300, 12, 5, nullptr, nullptr, &rp, part.data(), col.data(), b.data()) == FCLSH_EINVAL);
    std::vector<int32_t> sp(140214), sc(140214);
    std::vector<uint64_t> sb(140214);
    CHECK(fclsh_derive_params(140214, 13, 5, nullptr, &t, &rp, sp.data(), sc.data(), sb.data()) == FCLSH_OK);
    CHECK(t == 2 && rp == 6);

    // argument checks that return before any device work
    fclsh_index idx = nullptr;
    CHECK(fclsh_build_index(nullptr, 10, 64, 3, 1, nullptr, nullptr, &idx) == FCLSH_EINVAL && idx == nullptr);
    CHECK(fclsh_build_index(nullptr, 10, 5000, 3, 1, nullptr, nullptr, &idx) == FCLSH_EUNSUPPORTED);
    CHECK(fclsh_build_index_sparse(nullptr, nullptr, 10, 0, 5000, 3, 1, nullptr, nullptr, &idx) == FCLSH_EINVAL);
    CHECK(fclsh_build_index_sparse(nullptr, nullptr, 10, 0, kMaxSparseDims + 1, 3, 1, nullptr, nullptr, &idx) ==
          FCLSH_EUNSUPPORTED);
    int64_t total = 0;
    uint64_t offs[2];
    CHECK(fclsh_query_batch(nullptr, nullptr, 0, 0, nullptr, offs, nullptr, 0, &total) == FCLSH_EINVAL);
    CHECK(fclsh_query_batch_sparse(nullptr, nullptr, nullptr, 0, 0, 0, nullptr, offs, nullptr, 0, &total) ==
          FCLSH_EINVAL);
    CHECK(fclsh_hash(nullptr, nullptr, 0, nullptr, nullptr) == FCLSH_EINVAL);
    CHECK(fclsh_index_info(nullptr, nullptr, nullptr, nullptr, nullptr, nullptr, nullptr, nullptr, nullptr) ==
          FCLSH_EINVAL);
    fclsh_index_free(nullptr);
    fclsh_graph_free(nullptr);
    CHECK(std::strlen(fclsh_last_error()) > 0);
}

// Every piece of a carved workspace lies inside the buffer, and no two
// overlap.
static void workspace_layout() {
    const size_t sizes[] = {0, 100, 4096, size_t(1) << 20, size_t(64) << 20};
    const int64_t nqs[] = {0, 1, 7, 1000, 100000};
    const int Ls[] = {1, 31, 254, 4095};
    for (size_t bytes : sizes) {
        std::vector<unsigned char> buf(bytes + 1);
        char *base = reinterpret_cast<char *>(buf.data());
        for (int64_t nq : nqs)
            for (int L : Ls) {
                QueryWorkspace ws;
                const fclsh_status s = ws_carve(ws, base, bytes, nq, L);
                if (s != FCLSH_OK) {
                    CHECK(s == FCLSH_ENOMEM);
                    continue;
                }
                struct Piece {
                    const void *p;
                    size_t n;
                } pieces[] = {{ws.qkeys, size_t(std::max<int64_t>(nq * L, 1)) * 4},
                              {ws.qcount, size_t(nq + 1) * 4},
                              {ws.qfill, size_t(nq + 1) * 4},
                              {ws.qcount64, size_t(nq + 1) * 8},
                              {ws.scan_part, size_t(scan_partials_needed(nq + 1)) * 8},
                              {ws.ctrl, sizeof(QueryCtrl)},
                              {ws.spill, size_t(ws.cap_spill) * 16},
                              {ws.pq, size_t(ws.cap_pairs) * 4},
                              {ws.pid, size_t(ws.cap_pairs) * 4},
                              {ws.sorttmp, size_t(ws.cap_pairs) * 4}};
                for (const Piece &a : pieces) {
                    const char *pa = static_cast<const char *>(a.p);
                    CHECK(pa >= base && pa + a.n <= base + bytes);
                    CHECK((reinterpret_cast<uintptr_t>(pa) - reinterpret_cast<uintptr_t>(base)) % 256 == 0);
                    for (const Piece &c : pieces) {
                        if (&a == &c) continue;
                        const char *pc = static_cast<const char *>(c.p);
                        CHECK(pa + a.n <= pc || pc + c.n <= pa);
                    }
                }
                CHECK(ws.cap_pairs >= 1 && ws.cap_spill >= 1 && ws.cap_q == nq + 1 && ws.cap_items == nq * L);
                CHECK(ws_bytes(ws) > 0);
            }
    }
}

static void table_sizing() {
    const int64_t ns[] = {1, 2, 255, 256, 4097, 100000, 1000000, 4000000, 10000000, 100000000, 0x7FFFFFFF};
    for (int64_t n : ns) {
        const int db = table_dir_bits(n);
        CHECK(db >= 8 && db <= 19);
        const int sb = table_split_bits(n, db), mb = table_merge_bits(n, db);
        CHECK(sb >= 0 && mb >= 0 && sb + 8 - mb >= 1);
        // 6-byte entries only where 16-bit keys are stored, no groups are
        // merged (the key word then holds every key bit pass 2 reads) and the
        // ids fit 9 + 16 bits
        const bool pk = table_packed_pass1(n, db);
        CHECK(!pk || (table_key_bytes(db) == 2 && 31 - db <= 16 && mb == 0 && n <= (int64_t(1) << 25)));
        CHECK(pk == (table_key_bytes(db) == 2 && mb == 0 && n <= (int64_t(1) << 25)));
        for (int64_t L : {int64_t(1), int64_t(254), int64_t(4094), int64_t(65535)}) {
            const size_t s = table_build_scratch_bytes(L, n, db);
            CHECK(s > 0 && s < (size_t(1) << 62));
        }
    }
    for (int64_t n : {int64_t(0), int64_t(1), int64_t(255), int64_t(256), int64_t(1) << 40})
        CHECK(scan_partials_needed(n) >= 1);
}

int main() {
    params_grid();
    malformed_params();
    entry_point_arguments();
    workspace_layout();
    table_sizing();
    if (g_fail) {
        std::printf("%d checks failed\n", g_fail);
        return 1;
    }
    std::printf("library host checks passed\n");
    return 0;
}
