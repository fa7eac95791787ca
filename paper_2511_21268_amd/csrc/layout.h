// Constants of the device matrix layout shared by the kernels (HIP) and the
// host code that builds and checks the images (plain C++).
#pragma once

namespace amgk {
constexpr int WIN_LMAX = 7;      // longest offset run one staged x window covers
constexpr int WIN_ROWS = 64 + WIN_LMAX - 1;   // rows of one staged x window
}  // namespace amgk
