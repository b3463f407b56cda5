// Sub-panel width W and waves per SIMD of the LU panel kernel per precision,
// workgroup size and rows per thread R: "W, WPE" for each case.  Written by
// paper_1807_02718_amd/tune.py, which times every spill-free candidate on
// kite solves at N = 1024 and 4096 and keeps the fastest; edit by rerunning it.
#pragma once

// 256 threads (batches of more than 256 matrices), rows per thread R
#define FHW_PT_F32_256_R1 8, 4
#define FHW_PT_F32_256_R2 8, 4
#define FHW_PT_F32_256_R4 8, 4
#define FHW_PT_F64_256_R1 8, 4
#define FHW_PT_F64_256_R2 8, 2
#define FHW_PT_F64_256_R4 8, 2
// 1024 threads (batches of at most 256 matrices), rows per thread R
#define FHW_PT_F32_1024_R1 8, 4
#define FHW_PT_F32_1024_R2 8, 4
#define FHW_PT_F32_1024_R4 8, 4
#define FHW_PT_F64_1024_R1 8, 4
#define FHW_PT_F64_1024_R2 4, 4
#define FHW_PT_F64_1024_R4 4, 4
