// Particle checkpoint file (see checkpoint_host.hpp for the layout).
#include "checkpoint_host.hpp"

#include <unistd.h>

#include <algorithm>
#include <cerrno>
#include <cstdio>
#include <cstring>
#include <vector>

namespace etpic {
namespace ckpt {

uint64_t fnv1a(const void *p, size_t len, uint64_t h) {
    const unsigned char *b = static_cast<const unsigned char *>(p);
    for (size_t i = 0; i < len; ++i) {
        h ^= b[i];
        h *= 1099511628211ull;
    }
    return h;
}

uint64_t mesh_hash(int64_t n_vert, const double *xyz, int64_t n_tet, const int32_t *tet_vert) {
    uint64_t h = fnv1a(&n_vert, sizeof n_vert);
    h = fnv1a(&n_tet, sizeof n_tet, h);
    if (n_vert > 0 && xyz) h = fnv1a(xyz, sizeof(double) * 3 * (size_t)n_vert, h);
    if (n_tet > 0 && tet_vert) h = fnv1a(tet_vert, sizeof(int32_t) * 4 * (size_t)n_tet, h);
    return h;
}

size_t array_bytes(uint32_t precision, int64_t n, int k, bool has_id) {
    if (n < 0 || precision > 2 || k < 0 || k >= kArrays) return 0;
    const size_t m = (size_t)n;
    if (k == 0) return 4 * m;
    if (k <= 3) return (precision == 2 ? 4 : 8) * m;
    if (k <= 6) return (precision == 0 ? 8 : 4) * m;
    return has_id ? 8 * m : 0;
}

namespace {

uint64_t header_sum(Header h) {
    h.header_sum = 0;
    return fnv1a(&h, sizeof h);
}

std::string sys_error(const char *what, const std::string &path) {
    return std::string(what) + " " + path + ": " + std::strerror(errno);
}

struct File {
    FILE *f = nullptr;
    ~File() {
        if (f) std::fclose(f);
    }
};

}  // namespace

std::string write(const std::string &path, Header h, const Transfer &fetch, size_t chunk) {
    if (h.n < 0 || h.n > kMaxN) return "particle count out of range";
    if (h.precision > 2) return "bad precision";
    if (chunk == 0) return "zero chunk size";
    std::memcpy(h.magic, kMagic, sizeof kMagic);
    h.version = kVersion;
    h.reserved = 0;
    const std::string tmp = path + ".tmp";
    File out;
    out.f = std::fopen(tmp.c_str(), "wb");
    if (!out.f) return sys_error("cannot create", tmp);
    // on any failure the temporary file goes and an existing checkpoint stays
    auto abandon = [&](std::string e) {
        std::fclose(out.f);
        out.f = nullptr;
        std::remove(tmp.c_str());
        return e;
    };
    std::vector<unsigned char> buf(chunk);
    Header blank{};
    if (std::fwrite(&blank, sizeof blank, 1, out.f) != 1) return abandon(sys_error("cannot write", tmp));
    for (int k = 0; k < kArrays; ++k) {
        const size_t total = array_bytes(h.precision, h.n, k, h.has_id != 0);
        uint64_t s = kFnvOffset;
        for (size_t off = 0; off < total; off += chunk) {
            const size_t len = std::min(chunk, total - off);
            std::string e = fetch(k, off, buf.data(), len);
            if (!e.empty()) return abandon(e);
            s = fnv1a(buf.data(), len, s);
            if (std::fwrite(buf.data(), 1, len, out.f) != len) return abandon(sys_error("cannot write", tmp));
        }
        h.sums[k] = s;
    }
    h.header_sum = header_sum(h);
    if (std::fseek(out.f, 0, SEEK_SET) != 0 || std::fwrite(&h, sizeof h, 1, out.f) != 1)
        return abandon(sys_error("cannot write", tmp));
    if (std::fflush(out.f) != 0 || fsync(fileno(out.f)) != 0) return abandon(sys_error("cannot flush", tmp));
    const int rc = std::fclose(out.f);
    out.f = nullptr;
    if (rc != 0) {
        std::remove(tmp.c_str());
        return sys_error("cannot close", tmp);
    }
    if (std::rename(tmp.c_str(), path.c_str()) != 0) {
        std::string e = sys_error("cannot rename to", path);
        std::remove(tmp.c_str());
        return e;
    }
    return "";
}

std::string read_header(const std::string &path, Header &h) {
    File in;
    in.f = std::fopen(path.c_str(), "rb");
    if (!in.f) return sys_error("cannot open", path);
    if (std::fread(&h, sizeof h, 1, in.f) != 1) return "short file (no complete header): " + path;
    if (std::memcmp(h.magic, kMagic, sizeof kMagic) != 0) return "not a particle checkpoint: " + path;
    if (h.version != kVersion) return "checkpoint format version " + std::to_string(h.version) + " unknown";
    if (h.header_sum != header_sum(h)) return "checkpoint header checksum mismatch: " + path;
    if (h.precision > 2) return "checkpoint precision " + std::to_string(h.precision) + " unknown";
    if (h.n < 0 || h.n > kMaxN) return "checkpoint particle count " + std::to_string(h.n) + " out of range";
    size_t want = sizeof h;
    for (int k = 0; k < kArrays; ++k) want += array_bytes(h.precision, h.n, k, h.has_id != 0);
    if (std::fseek(in.f, 0, SEEK_END) != 0) return sys_error("cannot seek", path);
    const long got = std::ftell(in.f);
    if (got < 0 || (size_t)got != want)
        return "checkpoint size " + std::to_string(got) + " bytes, header announces " + std::to_string(want);
    return "";
}

std::string read(const std::string &path, const Header &h, const Transfer &store, size_t chunk) {
    if (chunk == 0) return "zero chunk size";
    File in;
    in.f = std::fopen(path.c_str(), "rb");
    if (!in.f) return sys_error("cannot open", path);
    if (std::fseek(in.f, (long)sizeof(Header), SEEK_SET) != 0) return sys_error("cannot seek", path);
    std::vector<unsigned char> buf(chunk);
    for (int k = 0; k < kArrays; ++k) {
        const size_t total = array_bytes(h.precision, h.n, k, h.has_id != 0);
        uint64_t s = kFnvOffset;
        for (size_t off = 0; off < total; off += chunk) {
            const size_t len = std::min(chunk, total - off);
            if (std::fread(buf.data(), 1, len, in.f) != len) return "short read of " + path;
            s = fnv1a(buf.data(), len, s);
            std::string e = store(k, off, buf.data(), len);
            if (!e.empty()) return e;
        }
        if (s != h.sums[k]) return "checkpoint array " + std::to_string(k) + " checksum mismatch: " + path;
    }
    return "";
}

}  // namespace ckpt
}  // namespace etpic
