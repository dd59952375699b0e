// rd_kernels.h -- host launchers of the pipeline stages (each defined in its own .hip file).
#pragma once
#include "rd_internal.h"

namespace rd {
void fill_u32(u32 *p, u64 n, u32 v, hipStream_t s);
void fill_u8(uint8_t *p, u64 n, uint8_t v, hipStream_t s);
void fill_u32_dyn(u32 *p, const u32 *count, u32 v, u64 max_n, hipStream_t s);
void scan_exclusive(u32 *data, u64 n, u32 *part, hipStream_t s);

void prep_init(const Bufs &b, hipStream_t s);
void prep_ingest(const Bufs &b, u64 *sync_mask, u64 *acc_mask, u64 *atom_mask, hipStream_t s);
void prep_sync_lists(const Bufs &b, const u64 *sync_mask, const u64 *atom_mask, hipStream_t s);
void prep_elements(const Bufs &b, const u64 *acc_mask, hipStream_t s);
void prep_thread_sync(const Bufs &b, u32 *rt_scan, hipStream_t s);
void prep_validate_wbar(const Bufs &b, hipStream_t s);

// knowledge vectors (releases, acquires, warp barriers)
void interp_run(const Bufs &b, const u32 *rt_scan, hipStream_t s);

// radix sort of the access elements by location key; returns nothing, sets the device-side
// buffer choice through Bufs::sorted_buf (fixed by the number of passes)
void sort_elements(const Bufs &b, hipStream_t s);
void sort_pairs(const Bufs &b, hipStream_t s);

void segcheck_run(const Bufs &b, const u32 *rt_scan, hipStream_t s);
}  // namespace rd
