// internal.hpp -- calls between the library's own translation units (not part
// of the C ABI): the served-labeling code batches small requests into shared
// launches through these, and the cubic-lattice sweep draws its initial
// states and records its errors through them.
#pragma once
#include <hip/hip_runtime.h>

#include <cstddef>
#include <cstdint>
#include <vector>

#include "../../include/swccl.h"

namespace swccl_internal {

// One labeling request of a batched launch: its input and outputs (device)
// and its own labeling workspace of ccl_workspace_bytes(W, H, mode) bytes.
struct LabelRequest {
    const uint8_t *in;
    int32_t W, H;
    int32_t *labels, *roots, *sizes, *n_clusters;
    void *ws;
};

// Tiles of one W x H request at the default tile shape.
int64_t request_tiles(int32_t W, int32_t H);

// Device table bytes a batch of n requests with ntiles tiles in all needs.
size_t batch_table_bytes(int32_t n, int64_t ntiles);

// Enqueue the labeling of n requests (one mode; with sizes iff `sizes`) as one
// launch per phase on stream s.  `table` is device memory and `stage` host
// memory (pinned, so the copy is asynchronous), each of at least
// batch_table_bytes(n, ntiles) <= table_bytes bytes; the table is written to
// `stage` and copied from there, so `stage` must stay unchanged until the
// stream has passed this call.
sw_status label_batch(const LabelRequest *r, int32_t n, int32_t mode, bool sizes, void *table, void *stage,
                      size_t table_bytes, hipStream_t s);

// SW_ERR_DEVICE with the message of e recorded for sw_last_error (SW_OK if
// e is hipSuccess).
sw_status device_error(hipError_t e, const char *where);

// Initial states of N sites: state_i = (w q) >> 32, w = word i&3 of
// Philox(i>>2, 0, INIT, sid), stored 0..q-1 or as Ising -1/+1.
sw_status init_spins(uint8_t *spins, int64_t N, int32_t q, bool ising, uint64_t seed, uint32_t sid, hipStream_t s);

// T = floor((1 - exp(-K)) 2^32), as sw_threshold.
uint64_t bond_threshold(double K);

// Enqueue a copy of n bytes from device-readable host memory (src_dev, the
// device address of pinned memory) to device memory as a kernel on stream s.
sw_status pull(void *dst, const void *src_dev, int64_t n, hipStream_t s);

}  // namespace swccl_internal
