// Launch layout of the blend shared by the host and the kernels.
#pragma once

namespace pv {

// Blocks per tile of kBlendTile probes: each block blends half the texel
// rows of its tile (four of the tile's eight wavefronts).
constexpr int kBlendSplit = 2;

}  // namespace pv
