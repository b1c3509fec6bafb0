// Exercise of the library's host-side C++ (mesh canonicalisation, start grid,
// tree-cotree split, field and Gauss-law system assembly, the particle
// checkpoint file) built with
// AddressSanitizer and UndefinedBehaviorSanitizer on the CPU.  Meshes are
// jittered Kuhn boxes made here; every call's output is checked for the
// invariants it must satisfy, and the rejection paths are driven with bad
// meshes.  Exit status 0 when everything holds.
#include <cmath>
#include <cstdint>
#include <cstdio>
#include <cstring>
#include <string>
#include <unistd.h>
#include <vector>

#include "checkpoint_host.hpp"
#include "field_host.hpp"
#include "mesh_host.hpp"

namespace {

int failures = 0;
void check(bool ok, const char *what, long long a = 0, long long b = 0) {
    if (!ok) {
        std::fprintf(stderr, "FAILED: %s (%lld, %lld)\n", what, a, b);
        ++failures;
    }
}

uint64_t lcg = 88172645463325252ull;
double uniform() {   // xorshift64, [0, 1)
    lcg ^= lcg << 13;
    lcg ^= lcg >> 7;
    lcg ^= lcg << 17;
    return (double)(lcg >> 11) * (1.0 / 9007199254740992.0);
}

// n[0] x n[1] x n[2] cells, 6 tets per cell (one per axis order), interior
// vertices jittered by up to 10 % of the spacing, rows ascending.
void kuhn(const int n[3], std::vector<double> &xyz, std::vector<int32_t> &tv) {
    const int nx = n[0] + 1, ny = n[1] + 1, nz = n[2] + 1;
    xyz.assign((size_t)nx * ny * nz * 3, 0.0);
    auto vid = [&](int i, int j, int k) { return (int32_t)((k * ny + j) * nx + i); };
    for (int k = 0; k < nz; ++k)
        for (int j = 0; j < ny; ++j)
            for (int i = 0; i < nx; ++i) {
                const int c[3] = {i, j, k};
                for (int d = 0; d < 3; ++d) {
                    double x = (double)c[d] / n[d];
                    if (c[d] > 0 && c[d] < n[d]) x += (uniform() - 0.5) * 0.2 / n[d];
                    xyz[3 * vid(i, j, k) + d] = x;
                }
            }
    const int perms[6][3] = {{0, 1, 2}, {0, 2, 1}, {1, 0, 2}, {1, 2, 0}, {2, 0, 1}, {2, 1, 0}};
    tv.clear();
    for (int k = 0; k < n[2]; ++k)
        for (int j = 0; j < n[1]; ++j)
            for (int i = 0; i < n[0]; ++i)
                for (auto &p : perms) {
                    int c[3] = {i, j, k};
                    int32_t v[4];
                    v[0] = vid(c[0], c[1], c[2]);
                    for (int s = 0; s < 3; ++s) {
                        c[p[s]] += 1;
                        v[s + 1] = vid(c[0], c[1], c[2]);
                    }
                    // ascending order
                    for (int a = 0; a < 4; ++a)
                        for (int b = a + 1; b < 4; ++b)
                            if (v[b] < v[a]) std::swap(v[a], v[b]);
                    tv.insert(tv.end(), v, v + 4);
                }
}

void exercise(const int n[3]) {
    std::vector<double> xyz;
    std::vector<int32_t> tv;
    kuhn(n, xyz, tv);
    const int64_t nv = (int64_t)xyz.size() / 3, nt = (int64_t)tv.size() / 4;
    etpic::HostMesh M;
    std::string err;
    const int rc = etpic::build_host_mesh(nv, xyz.data(), nt, tv.data(), M, err);
    check(rc == 0, "build_host_mesh", rc);
    if (rc) return;
    check(M.nv - M.ne + M.nf - M.nt == 1, "Euler characteristic of a ball", M.nv - M.ne + M.nf - M.nt);
    check((int64_t)M.e2s_slot.size() == 6 * nt, "edge -> slot CSR size");
    check(M.e2s_ptr.back() == 6 * nt, "edge -> slot CSR end", M.e2s_ptr.back());
    check(M.v2e_ptr.back() == 2 * M.ne, "vertex -> edge CSR end", M.v2e_ptr.back());
    etpic::StartGrid g;
    etpic::build_start_grid(M, xyz.data(), 2.0, g);
    for (int32_t t : g.cell) check(t >= 0 && t < nt, "start tet in range", t);
    std::vector<uint8_t> et((size_t)M.ne), ft((size_t)M.nf);
    etpic::tree_cotree(M, et.data(), ft.data());
    int64_t te = 0, tf = 0;
    for (uint8_t b : et) te += b;
    for (uint8_t b : ft) tf += b;
    check(te == M.nv - 1, "spanning tree of the vertices", te, M.nv - 1);
    check(tf == M.nt, "spanning tree of tets + exterior", tf, M.nt);
    for (int dir = 0; dir < 2; ++dir) {
        etpic::FieldSystem F;
        const int fr = etpic::build_field_system(M, 8.85e-12, 1.2566e-6, F, err, dir == 0);
        check(fr == 0, "build_field_system", fr);
        if (fr) continue;
        check(F.rowptr.back() == F.nnz, "field CSR end");
        for (int64_t i = 0; i < F.ne; ++i)
            for (int32_t j = F.rowptr[i]; j < F.rowptr[i + 1]; ++j)
                check(F.col[j] >= 0 && F.col[j] < F.ne && std::isfinite(F.M[j]) && std::isfinite(F.K[j]),
                      "field entry", i, j);
    }
    etpic::NsSystem S;
    const int nr = etpic::build_ns_system(M, 8.85e-12, S, err);
    check(nr == 0, "build_ns_system", nr);
    if (!nr) {
        // rows of inner nodes none of whose neighbours is a wall node kill
        // constants (the stiffness of linear elements); the matrix is
        // symmetric with a positive diagonal
        double rowsum = 0.0, scale = 0.0, asym = 0.0;
        for (int64_t i = 0; i < S.nv; ++i) {
            bool wall_near = S.wall[i] != 0;
            for (int32_t k = M.v2e_ptr[i]; k < M.v2e_ptr[i + 1]; ++k) {
                const int32_t e = M.v2e_code[k] >> 1;
                const int32_t w = (M.v2e_code[k] & 1) ? M.edges[2 * e] : M.edges[2 * e + 1];
                if (S.wall[w]) wall_near = true;
            }
            double r = 0.0, d = 0.0;
            for (int32_t j = S.rowptr[i]; j < S.rowptr[i + 1]; ++j) {
                r += S.S[j];
                scale = std::max(scale, std::fabs(S.S[j]));
                if (S.col[j] == i) d = S.S[j];
                // the transposed entry
                const int32_t c = S.col[j];
                double t = 0.0;
                for (int32_t q = S.rowptr[c]; q < S.rowptr[c + 1]; ++q)
                    if (S.col[q] == i) t = S.S[q];
                asym = std::max(asym, std::fabs(t - S.S[j]));
            }
            check(d > 0.0, "positive diagonal", i);
            if (!wall_near) rowsum = std::max(rowsum, std::fabs(r));
        }
        check(rowsum <= 1e-9 * scale, "stiffness kills constants at inner nodes");
        check(asym <= 1e-12 * scale, "stiffness symmetric");
    }
}

void rejections() {
    std::string err;
    const double xyz[] = {0, 0, 0, 1, 0, 0, 0, 1, 0, 0, 0, 1, 1, 1, 1, 0.2, 0.2, -1, 0.3, 0.3, 2.0};
    etpic::HostMesh M;
    const int32_t unsorted[] = {0, 2, 1, 3};
    check(etpic::build_host_mesh(7, xyz, 1, unsorted, M, err) != 0, "unsorted row refused");
    const int32_t out_of_range[] = {0, 1, 2, 9};
    check(etpic::build_host_mesh(7, xyz, 1, out_of_range, M, err) != 0, "vertex out of range refused");
    const double flat[] = {0, 0, 0, 1, 0, 0, 0, 1, 0, 1, 1, 0};
    const int32_t one[] = {0, 1, 2, 3};
    check(etpic::build_host_mesh(4, flat, 1, one, M, err) != 0, "flat tet refused");
    const int32_t three[] = {0, 1, 2, 3, 0, 1, 2, 5, 0, 1, 2, 6};
    check(etpic::build_host_mesh(7, xyz, 3, three, M, err) != 0, "non-manifold face refused");
}

// Particle checkpoint: write from host arrays and read back through small
// chunks (so that arrays span several), every precision with and without ids;
// a corrupted array byte, a truncated file and a failing transfer are
// reported, and a failed write leaves the previous checkpoint in place.
void checkpoints(const std::string &dir) {
    namespace ck = etpic::ckpt;
    const std::string path = dir + "/host_driver_ckpt.bin";
    for (uint32_t prec = 0; prec <= 2; ++prec)
        for (int has_id = 0; has_id <= 1; ++has_id) {
            const int64_t n = 1003;
            std::vector<std::vector<unsigned char>> src(ck::kArrays), dst(ck::kArrays);
            for (int k = 0; k < ck::kArrays; ++k) {
                src[k].resize(ck::array_bytes(prec, n, k, has_id != 0));
                for (auto &b : src[k]) b = (unsigned char)(uniform() * 256.0);
                dst[k].assign(src[k].size(), 0);
            }
            ck::Header h{};
            h.precision = prec;
            h.n = n;
            h.step = 77;
            h.n_tet = 5;
            h.n_vert = 9;
            h.mesh_hash = 42;
            h.has_id = (uint32_t)has_id;
            auto fetch = [&](int k, size_t off, void *buf, size_t len) -> std::string {
                if (off + len > src[k].size()) return "fetch out of range";
                std::memcpy(buf, src[k].data() + off, len);
                return "";
            };
            auto store = [&](int k, size_t off, void *buf, size_t len) -> std::string {
                if (off + len > dst[k].size()) return "store out of range";
                std::memcpy(dst[k].data() + off, buf, len);
                return "";
            };
            check(ck::write(path, h, fetch, 1000).empty(), "checkpoint written", prec, has_id);
            ck::Header r{};
            check(ck::read_header(path, r).empty(), "checkpoint header read", prec, has_id);
            check(r.n == n && r.step == 77 && r.precision == prec && r.has_id == (uint32_t)has_id &&
                      r.mesh_hash == 42,
                  "checkpoint header fields", prec, has_id);
            check(ck::read(path, r, store, 777).empty(), "checkpoint arrays read", prec, has_id);
            for (int k = 0; k < ck::kArrays; ++k) check(src[k] == dst[k], "checkpoint array round trip", k, prec);
            // a failing transfer: the write fails and the previous file stays
            auto broken = [&](int k, size_t, void *, size_t) -> std::string { return k == 5 ? "device gone" : ""; };
            check(!ck::write(path, h, broken, 1000).empty(), "failed write reported", prec);
            check(ck::read_header(path, r).empty(), "previous checkpoint intact", prec);
            FILE *t = std::fopen((path + ".tmp").c_str(), "rb");
            check(t == nullptr, "temporary file removed", prec);
            if (t) std::fclose(t);
        }
    // corruption of one array byte and truncation
    {
        ck::Header r{};
        check(ck::read_header(path, r).empty(), "header before corruption");
        FILE *f = std::fopen(path.c_str(), "r+b");
        check(f != nullptr, "open for corruption");
        if (f) {
            std::fseek(f, (long)sizeof(ck::Header) + 10, SEEK_SET);
            int c = std::fgetc(f);
            std::fseek(f, (long)sizeof(ck::Header) + 10, SEEK_SET);
            std::fputc(c ^ 0x40, f);
            std::fclose(f);
        }
        std::vector<unsigned char> sink(8 * 1003);
        auto store = [&](int, size_t off, void *buf, size_t len) -> std::string {
            if (off + len > sink.size()) return "store out of range";
            std::memcpy(sink.data() + off, buf, len);
            return "";
        };
        const std::string e = ck::read(path, r, store, 4096);
        check(e.find("checksum") != std::string::npos, "corrupted array detected");
        f = std::fopen(path.c_str(), "r+b");
        if (f) {
            std::fseek(f, 0, SEEK_END);
            const long len = std::ftell(f);
            std::fclose(f);
            check(truncate(path.c_str(), len - 3) == 0, "truncate");
        }
        check(!ck::read_header(path, r).empty(), "truncated file refused");
    }
    std::remove(path.c_str());
}

}  // namespace

int main(int argc, char **argv) {
    const int sizes[][3] = {{1, 1, 1}, {2, 3, 2}, {5, 4, 6}, {8, 8, 8}};
    for (auto &n : sizes) exercise(n);
    rejections();
    checkpoints(argc > 1 ? argv[1] : ".");
    if (failures) {
        std::fprintf(stderr, "%d check(s) failed\n", failures);
        return 1;
    }
    std::printf("host driver: all checks passed\n");
    return 0;
}
