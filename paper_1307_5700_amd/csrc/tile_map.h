// Workgroup -> (DM block, time tile) mapping of the dedispersion kernels.
#pragma once

#include <hip/hip_runtime.h>

namespace mbtp {

struct TileIdx {
  int dblock, ttile;
};

// Consecutive workgroups go to different XCDs (workgroup id mod 8); each
// XCD takes a contiguous range of tiles, DM block fastest, so the blocks
// that share a time tile run on the same L2 at about the same time.  When
// the last DM block is partial (`partial`: its idle consumers make its tiles
// cheaper), each XCD takes its share of the full blocks' tiles first and its
// share of the partial block's last, so the cheap tiles fill the final,
// partly occupied round.  A bijection from [0, nd*nt) onto the tiles.
__host__ __device__ inline TileIdx xcd_tile(int bid, int nd, int nt, bool partial) {
  const int ntile = nd * nt;
  const int xcd = bid & 7, slot = bid >> 3;
  const int q8 = ntile >> 3, rem = ntile & 7;
  TileIdx r;
  if (partial && nd > 1 && nt >= 8) {
    const int nfull = (nd - 1) * nt;
    const int f8 = nfull >> 3, frem = nfull & 7;
    const int nf = f8 + (xcd < frem ? 1 : 0);            // full tiles of this XCD
    const int fb = xcd * f8 + min(xcd, frem);            // first of them
    if (slot < nf) {
      r.dblock = (fb + slot) % (nd - 1);
      r.ttile = (fb + slot) / (nd - 1);
    } else {
      r.dblock = nd - 1;
      r.ttile = xcd * q8 + min(xcd, rem) - fb + (slot - nf);
    }
  } else {
    const int tile = xcd * q8 + min(xcd, rem) + slot;
    r.dblock = tile % nd;
    r.ttile = tile / nd;
  }
  return r;
}

}  // namespace mbtp
