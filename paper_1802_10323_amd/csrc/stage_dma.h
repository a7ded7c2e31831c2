// stage_dma.h - reading a tile of lines straight from global memory into a
// staging area of LDS (global_load_lds), for kernels that transform or
// eliminate one tile while the next one is in flight.
//
// The stage holds the tile as it lies in memory: strided layout, NL values
// of each point's row (row-major, NL per row); contiguous layout, the tile's
// run of NL lines of N values.  Each lane moves one 16-byte piece per
// instruction, so a piece must not straddle two lines of different rows
// (strided: rows of NL values split into whole pieces, the x extent a
// multiple of the piece); pieces outside the field read the field's first
// bytes instead and are never used.
#pragma once
#include "device_common.h"

namespace poisson_dev {

// One 16-byte piece per lane from global memory straight into LDS: lane i of
// the wave writes bytes [16 i, 16 i + 16) after `lds_addr` (wave-uniform).
// Inline assembly, so that the compiler does not treat it as an LDS write
// that later LDS accesses must wait for (it cannot tell the stage from the
// rest of LDS); the kernel waits for it explicitly (s_waitcnt) before
// reading the stage.
__device__ __forceinline__ void stage_dma16(const void* gaddr, unsigned lds_addr) {
  asm volatile(
      "s_mov_b32 m0, %1\n\t"
      "global_load_lds_dwordx4 %0, off"
      :
      : "v"(gaddr), "s"(__builtin_amdgcn_readfirstlane(lds_addr))
      : "memory", "m0");
}

template <typename T, int NL, int N>
struct StageLayout {
  static constexpr int EPL = 16 / (int)sizeof(T);              // values per piece
  static constexpr int BYTES = NL * N * (int)sizeof(T);
  static constexpr int CHUNKS = BYTES / 1024;                  // one wave instruction each
  static constexpr int PER_WAVE = (CHUNKS + 7) / 8;            // 512 threads = 8 waves
  static constexpr int LANES_PER_ROW = NL / EPL;
  static constexpr int ROWS_PER_CHUNK = 64 / LANES_PER_ROW;
  static_assert(BYTES % 1024 == 0, "the stage is whole 1 KiB chunks");
  static_assert(NL % EPL == 0 && 64 % LANES_PER_ROW == 0, "rows of whole pieces");
};

// Issue the reads of tile `tile` (lines of n = N points described by g) into
// the stage.  Completion is awaited by the vector-memory counter.
template <typename T, int NL, int N>
__device__ __forceinline__ void stage_fetch(lptr<unsigned char> stage, const T* data,
                                            const LineGeom& g, int tile, int tid) {
  using SL = StageLayout<T, NL, N>;
  const TileOrigin o = tile_origin(g, tile);
  const int wave = tid >> 6, lane = tid & 63;
  const int nlt = 1 << g.lognl;
#pragma unroll
  for (int j = 0; j < SL::PER_WAVE; ++j) {
    const int c = wave * SL::PER_WAVE + j;     // chunk of this instruction (wave-uniform)
    if (c < SL::CHUNKS) {
      const T* src = data;
      if (g.layout == 0) {
        const int row = c * SL::ROWS_PER_CHUNK + lane / SL::LANES_PER_ROW;
        const int l = (lane % SL::LANES_PER_ROW) * SL::EPL;
        const long long b = l < nlt ? line_base(g, o, l) : -1;
        if (b >= 0) src = data + b + (long long)row * g.sp;
      } else {
        const int e = (c * 64 + lane) * SL::EPL;
        if (e / N < g.nlines - o.L0 && e / N < nlt) src = data + (long long)o.L0 * N + e;
      }
      stage_dma16(src, (unsigned)(size_t)(stage + c * 1024));
    }
  }
}

}  // namespace poisson_dev
