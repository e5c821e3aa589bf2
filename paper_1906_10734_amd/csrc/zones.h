// The 6^3 block of level-l cube positions around a parent of targets (Sec. 2.1), used by the
// enumeration of cubes that lie inside coarser leaves and by the per-parent source tables.
//
// A target T at level l >= 2 with parent P sees the 6^3 block of level-l cubes around P: block
// cube b = (bx, by, bz) in [0, 6)^3 sits at integer position 2 (P - 1) + b. The 27 cubes within
// distance one of T are its near zone; the other 189 are its interaction zone. On an adaptive
// tree a cube position is either a real level-l cell, a child position of a level-(l-1) leaf, or
// lies inside a coarser leaf: those last two are "virtual" cubes, whose effective masses come
// from the particles they contain (Eq. 5), so the zones partition space exactly at every level.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "dev_common.h"

namespace hpm {

struct IzSlot {
  int real;      // >= 0: the real level-l cell at this position
  int coarse;    // >= 0: the coarser leaf that holds the (virtual) cube
  uint32_t key;  // Morton key of the cube at level l (valid when coarse >= 0)
};

// Cube "slot" (< 216, x fastest) of the 6^3 block around parent P = (px, py, pz) at level l - 1
// (cell id par): the level-l position 2 (P - 1) + b. nbr27[par] encodes the 27 level-(l-1)
// positions around the parent: >= 0 a real cell, -1 empty, <= -2 inside the coarser leaf
// -2 - e. flags bit 0 marks a cell with children.
__device__ __forceinline__ IzSlot block_cube(int px, int py, int pz, int l, int par, int slot,
                                             const int* nbr27, const int* flags, const int* child8) {
  IzSlot r{-1, -1, 0u};
  const int bx = slot % 6, by = (slot / 6) % 6, bz = slot / 36;
  const int e = nbr27[par * 27 + (bx >> 1) + 3 * (by >> 1) + 9 * (bz >> 1)];
  const int oct = (bx & 1) | ((by & 1) << 1) | ((bz & 1) << 2);
  int coarse = -1;
  if (e >= 0) {
    if (flags[e] & 1) r.real = child8[e * 8 + oct];
    else coarse = e;
  } else if (e <= -2) {
    coarse = -2 - e;
  }
  if (coarse >= 0) {
    const int qx = 2 * (px - 1) + bx, qy = 2 * (py - 1) + by, qz = 2 * (pz - 1) + bz;
    r.coarse = coarse;
    r.key = morton3(uint32_t(qx), uint32_t(qy), uint32_t(qz), l);
  }
  return r;
}

// A cube's identifier across levels: its level-l Morton key below a leading 1 bit at 3 l
// (l <= 10, so it fits in 31 bits and ids of different levels never coincide).
__device__ __forceinline__ uint32_t cube_id(int l, uint32_t key) { return (1u << (3 * l)) | key; }
__device__ __forceinline__ int cube_id_level(uint32_t id) { return (31 - __clz(int(id))) / 3; }

}  // namespace hpm
