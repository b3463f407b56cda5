// K-chunk GK (staged through LDS) and workgroups per CU (launch-bounds hint)
// of the LU trailing-update / TRSM GEMM kernel per precision.  Written by
// paper_1807_02718_amd/tune.py (gemm mode), which times every spill-free
// candidate on the kite batch at N = 1024 (and, in FP64, a star-curve batch)
// and keeps the fastest; edit by rerunning it.
#pragma once

#define FHW_GEMM_GK_F32 16
#define FHW_GEMM_OCC_F32 4
#define FHW_GEMM_GK_F64 16
#define FHW_GEMM_OCC_F64 2
