// One tile shape of the persistent scoring kernel, every sink.  Compiled
// once per row of kTileShapes with -DSNCC_TILE_ENTRY_ID=<row>, so that the
// shapes build in parallel.
#include "tile_kernel.hpp"

#ifndef SNCC_TILE_ENTRY_ID
#error "compile with -DSNCC_TILE_ENTRY_ID=<row of kTileShapes>"
#endif

namespace sncc {

namespace {
constexpr int kRU = kTileShapes[SNCC_TILE_ENTRY_ID][0];
constexpr int kRV = kTileShapes[SNCC_TILE_ENTRY_ID][1];
constexpr int kNW = kTileShapes[SNCC_TILE_ENTRY_ID][2];
}  // namespace

#define SNCC_TILE_FN_(i) tile_fn_##i
#define SNCC_TILE_FN(i) SNCC_TILE_FN_(i)

const void *SNCC_TILE_FN(SNCC_TILE_ENTRY_ID)(int sink) {
  switch (sink) {
    case kSinkTopk: return reinterpret_cast<const void *>(&tile_kernel<kRU, kRV, kNW, kSinkTopk>);
    case kSinkMap: return reinterpret_cast<const void *>(&tile_kernel<kRU, kRV, kNW, kSinkMap>);
    default: return reinterpret_cast<const void *>(&tile_kernel<kRU, kRV, kNW, kSinkCompact>);
  }
}

}  // namespace sncc
