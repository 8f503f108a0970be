// Sweep-pass scheduler: groups the gate instances of a circuit into passes,
// each applying an order-preserving subset of gates that acts inside one tile
// of `nt` qubits.
#pragma once

#include <stdint.h>

#include <string>
#include <vector>

#include "rq_internal.h"

namespace rqk {

struct PlanPass {
  uint32_t qmask = 0;       // row bit positions of the tile
  int pos[8] = {0};         // row bit position of local bit b
  std::vector<GateRef> gates;
};

// k: qubits; pairs [n][2]; parity: qubit k-1 is implied (sector-compressed
// states); nt: tile qubits (explicit); maxg: gate cap per pass.
// Returns false and sets err on invalid input.
bool plan_passes(int k, int n, const int32_t *pairs, bool parity, int nt, int maxg,
                 std::vector<PlanPass> &out, std::string &err);

}  // namespace rqk
