// Layout of the per-device scratch array of chem_integrate_noalloc (noalloc.hip): the persistent
// kernels' work-queue counter, the probe/resume schedule (bin counts and offsets), the parked
// cells' continuation state and resume order, and the per-cell counters when the caller passes
// none.  Sized for up to kNoAllocMaxCells cells.
#pragma once
#include <hip/hip_runtime.h>

#include <cstddef>
#include <cstdint>

namespace chem_noalloc {
constexpr int64_t kMaxCells = int64_t(1) << 20;
constexpr size_t kQueueOff = 0;                                        // u64 queue counter
constexpr size_t kSchedOff = 256;                                      // u32 [2 + 2 * 256]
constexpr size_t kWstOff = 4352;                                       // f64 [4][n]
constexpr size_t kOrderOff = kWstOff + 4 * sizeof(double) * kMaxCells;  // i32 [n]
constexpr size_t kCountersOff = kOrderOff + sizeof(int) * kMaxCells;   // i32 [3][ld]
constexpr size_t kBytes = kCountersOff + 3 * sizeof(int) * kMaxCells;  // 48 MiB + 4352 B
static_assert(kWstOff % 256 == 0 && kOrderOff % 256 == 0 && kCountersOff % 256 == 0, "aligned parts");

// Device address of the scratch array on `device`, resolved with hipGetSymbolAddress once per
// device (with that device current) and cached; later calls return the cached address.
hipError_t scratch_address(int device, void** out);
}  // namespace chem_noalloc
