// csr7.h -- where the blocks of a cell sit in the caller's CSR layout of the
// 7-point pattern, in closed form.
//
// The pattern of an nx x ny x nz grid with blocks in ascending column order
// (-z, -y, -x, self, +x, +y, +z, those inside the grid) is unique, so a row
// start is a count: every earlier cell contributes its diagonal and one block
// per face it has.  rs_bsr_create checks the caller's row pointer against
// this count, so kernels reading the caller's values need neither the row
// pointer nor the column indices.  All counts fit in 32 bits (the library
// admits nnzb <= INT32_MAX).
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

struct csr7_row {
  uint32_t start;   // caller block index of the row's first block
  uint32_t mask;    // bit s set when slot s lies inside the grid
};

__device__ __forceinline__ csr7_row csr7_of(uint32_t c, uint32_t nx, uint32_t ny, uint32_t nz) {
  const uint32_t nxy = nx * ny;
  const uint32_t k = c / nxy, inp = c - k * nxy;   // plane, index within it
  const uint32_t j = inp / nx, i = inp - j * nx;
  const uint32_t line = k * ny + j;                 // complete x-lines before c
  uint32_t before = c;                              // diagonals
  before += 2 * line * (nx - 1) + (i > 0 ? 2 * i - 1 : 0);          // x faces
  const uint32_t yl = nx * (ny - 1);                                // y links per plane
  before += 2 * k * yl + (inp < yl ? inp : yl) + (inp > nx ? inp - nx : 0);
  const uint32_t zl = nxy * (nz - 1);                               // z links
  before += (c < zl ? c : zl) + (c > nxy ? c - nxy : 0);
  uint32_t m = 8u;
  m |= (k > 0 ? 1u : 0u) | (j > 0 ? 2u : 0u) | (i > 0 ? 4u : 0u);
  m |= (i + 1 < nx ? 16u : 0u) | (j + 1 < ny ? 32u : 0u) | (k + 1 < nz ? 64u : 0u);
  return {before, m};
}

// Caller block index of slot s of the row; an off-grid slot gives the row's
// diagonal block, a valid address whose value the caller replaces by zero.
__device__ __forceinline__ uint32_t csr7_pos(const csr7_row &w, int s) {
  const uint32_t below = w.mask & ((1u << s) - 1u);
  const uint32_t p = w.start + (uint32_t)__popc(below);
  const uint32_t pd = w.start + (uint32_t)__popc(w.mask & 7u);
  return ((w.mask >> s) & 1u) ? p : pd;
}
