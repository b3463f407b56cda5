// Sub-panel width W and waves per SIMD of the LU panel kernel per precision,
// workgroup size and rows per thread R: "W, WPE" (and, for large batches,
// the workgroup size) for each case.  Written by
// paper_1807_02718_amd/tune.py, which times every spill-free candidate on
// kite solves at N = 1024 and 4096 (tall panels: star-curve batches at
// N = 1536 and 4096) and keeps the fastest; edit by rerunning it.
#pragma once

// Batches of more than 256 matrices: "threads, W, WPE, PD" per precision and
// rows per 256 threads R (R = 1, 2, 4: panels of up to 256, 512, 1024 rows);
// a thread takes ceil(256 R / threads) rows; PD columns of each factored
// sub-panel in flight during the lazy updates (0: the kernel's default)
#define FHW_PB_F32_R1 256, 8, 4, 0
#define FHW_PB_F32_R2 256, 8, 2, 2
#define FHW_PB_F32_R4 256, 8, 4, 0
#define FHW_PB_F64_R1 256, 8, 2, 2
#define FHW_PB_F64_R2 256, 8, 2, 1
#define FHW_PB_F64_R4 256, 8, 2, 1
// tall panels of large batches: R = 8, 16 (up to 2048, 4096 rows)
#define FHW_PB_F32_R8 512, 4, 2, 0
#define FHW_PB_F32_R16 512, 8, 2, 0
#define FHW_PB_F64_R8 512, 8, 2, 0
#define FHW_PB_F64_R16 512, 4, 2, 0
// 1024 threads (batches of at most 256 matrices), rows per thread R
#define FHW_PT_F32_1024_R1 8, 4
#define FHW_PT_F32_1024_R2 8, 4
#define FHW_PT_F32_1024_R4 8, 4
#define FHW_PT_F64_1024_R1 8, 4
#define FHW_PT_F64_1024_R2 4, 4
#define FHW_PT_F64_1024_R4 4, 4
