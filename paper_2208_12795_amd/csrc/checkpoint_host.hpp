// Host-side particle checkpoint file: layout, checksums, chunked write and
// read.  No GPU code: the library moves each chunk between device and host
// through the callbacks, and the sanitizer driver exercises the format alone.
//
// File (little-endian): a 136-byte header, then the arrays in this order,
// each n elements, no padding:
//   tet int32; lam_1, lam_2, lam_3 (float64, or uint32 fixed point for the
//   compact mixed form); v_x, v_y, v_z (float64, or float32 for both mixed
//   forms); id int64 (only if has_id).
// The header holds the format version, precision, n, the step index, the
// mesh's tet and vertex counts and a hash of its vertex coordinates and tet
// vertex ids (a checkpoint resumes only on the mesh it was taken on), the
// FNV-1a 64-bit checksum of every array and of the header itself.
#pragma once
#include <cstddef>
#include <cstdint>
#include <functional>
#include <string>

namespace etpic {
namespace ckpt {

constexpr char kMagic[8] = {'E', 'T', 'P', 'I', 'C', 'C', 'K', 'P'};
constexpr uint32_t kVersion = 1;
constexpr int kArrays = 8;   // tet, lam 1..3, v 0..2, id
constexpr int64_t kMaxN = (int64_t)1 << 40;   // bound on n, so that no byte count overflows

struct Header {
    char magic[8];
    uint32_t version;
    uint32_t precision;   // 0 float64, 1 mixed, 2 compact mixed
    int64_t n;
    int64_t step;
    int64_t n_tet;
    int64_t n_vert;
    uint64_t mesh_hash;
    uint32_t has_id;
    uint32_t reserved;
    uint64_t sums[kArrays];
    uint64_t header_sum;   // FNV-1a of the header with this field zero
};
static_assert(sizeof(Header) == 136, "checkpoint header is 136 bytes");

constexpr uint64_t kFnvOffset = 1469598103934665603ull;
uint64_t fnv1a(const void *p, size_t len, uint64_t h = kFnvOffset);

// hash of a mesh as uploaded (vertex coordinates, tet vertex ids, counts)
uint64_t mesh_hash(int64_t n_vert, const double *xyz, int64_t n_tet, const int32_t *tet_vert);

// bytes of array k (0 tet, 1..3 lam, 4..6 v, 7 id) for n particles; 0 for an
// absent id array or a bad precision
size_t array_bytes(uint32_t precision, int64_t n, int k, bool has_id);

// Chunk transfer: moves `len` bytes at byte offset `off` of array k between
// the caller's storage and `buf`; returns 0 or an error message.
using Transfer = std::function<std::string(int k, size_t off, void *buf, size_t len)>;

// Writes the checkpoint of `h` (magic, version, checksums filled in here)
// to `path` through a temporary file renamed at the end, so that an existing
// checkpoint is replaced whole or not at all.  fetch copies chunks out of the
// particle arrays.  Returns "" or an error message.
std::string write(const std::string &path, Header h, const Transfer &fetch, size_t chunk = (size_t)16 << 20);

// Reads and validates the header of `path` (magic, version, header checksum,
// known precision, file size against the arrays it announces).
std::string read_header(const std::string &path, Header &h);

// Reads the arrays of `path` (whose header `h` read_header returned) chunk by
// chunk through store and checks every array's checksum.  On a checksum error
// the arrays have been partly overwritten.
std::string read(const std::string &path, const Header &h, const Transfer &store, size_t chunk = (size_t)16 << 20);

}  // namespace ckpt
}  // namespace etpic
