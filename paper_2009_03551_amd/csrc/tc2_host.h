// Host-side checks shared by the entry points of include/tc2.h.
#pragma once

#include <string>

#include "../../include/tc2.h"

namespace tc2 {

// A BSR matrix of nb x nb blocks of size b: ranges, strictly increasing
// columns per row, a symmetric pattern and finite values.
tc2_status validate_bsr(const tc2_bsr& m, int nb, int b);

// Every diagonal block is stored.
bool has_diag(const tc2_bsr& m, int nb);

// Make `device` current after checking that it exists and is a gfx950;
// its architecture name goes to *arch when arch is not NULL.
tc2_status select_gfx950(int device, std::string* arch);

}  // namespace tc2
