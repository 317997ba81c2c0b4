// Workgroup order across the 8 XCDs of an MI355X.
#pragma once

#include <hip/hip_runtime.h>

namespace smg {

// The hardware deals the workgroups of a launch to the 8 XCDs round robin
// (workgroup b to XCD b mod 8).  Returns the logical index that gives every
// XCD a contiguous range of logical indices (the first G mod 8 XCDs one more),
// so that neighbouring logical work shares one XCD's L2.  A bijection of
// [0, G) for every G >= 1.
__device__ inline int xcd_contiguous(int bid, int G) {
    const int xcd = bid & 7, local = bid >> 3;
    const int per = G >> 3, extra = G & 7;
    return xcd * per + (xcd < extra ? xcd : extra) + local;
}

}  // namespace smg
