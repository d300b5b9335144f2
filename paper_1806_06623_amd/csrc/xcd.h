// Workgroup order for stencil kernels over the (j, k) plane.
//
// The hardware hands workgroups to the 8 XCDs (each with its own L2) in turn:
// workgroup x runs on XCD x % 8.  A stencil kernel whose grid is gx blocks of
// the (j, k) plane per chunk of radial rows reads, besides its own block, the
// theta neighbours in the next and previous rows of the plane, which the
// neighbouring blocks load as their own.  With gx a multiple of 8 the plane
// blocks are permuted so that the workgroups of one XCD cover a contiguous
// range of the plane: a block's neighbours are then loaded into the same L2,
// at about the same time, instead of being fetched from HBM once more by
// another XCD.
#pragma once
#include <hip/hip_runtime.h>

__device__ __forceinline__ int spp_plane_block(int x, int gx)
{
    return gx % 8 == 0 ? (x % 8) * (gx / 8) + x / 8 : x;
}
