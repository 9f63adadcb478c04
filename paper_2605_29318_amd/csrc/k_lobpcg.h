// Row-chunk descriptors shared by the eigensolver kernels and their host code.
#pragma once
#include <cstdint>

namespace ff {
namespace lob {

// A run of rows of one object: resid/update work unit (<= 256 rows) or
// Gram partial-sum unit (<= 2048 rows). Chunks never straddle objects.
struct UChunk {
    int64_t r0;
    int32_t len;
    int32_t obj;
};
typedef UChunk GChunk;

}  // namespace lob
}  // namespace ff

struct ff_ctx;
namespace ff {
namespace lob {

// Once per device (the context's, current): the address of rayleigh_ritz_noalloc's fixed scratch.
int noalloc_setup(ff_ctx *ctx);

}  // namespace lob
}  // namespace ff
