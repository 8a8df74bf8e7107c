// Host geometry builder of libdd.
#pragma once

#include <cstdint>
#include <string>
#include <vector>

#include "dd_internal.h"

namespace dd {

// Fill the host tables of B from n boxes [n][8] (origin, extent) and optional
// inner boxes [n][8] (offset, extent).  With frames set, every block's solve
// domain is its box minus its inner box.  Returns "" or an error message.
std::string build_geometry(dd_blocks *B, const int L[4], int tbc, int n, const int32_t *boxes,
                           const int32_t *inner, bool frames = false);

// Fill the host tables of D as the inactive-region domain of B: one block,
// the whole lattice minus the union of B's inner boxes (their sites
// decoupled), the hops from those boxes into it as exterior hops, and the
// dPi_1 site list.  Returns "" or an error message.
std::string build_inactive(dd_blocks *D, const dd_blocks *B);

// 1 for every block site (block layout: blocks in order, eo slots within a
// block) that lies in its block's hole (a frame's inner box, or a masked
// site of an inactive-region domain), else 0; empty when no block has a hole.
std::vector<uint8_t> hole_slots(const dd_blocks *B);

}  // namespace dd
