// Constants of the device matrix layout shared by the kernels (HIP) and the
// host code that builds and checks the images (plain C++).
#pragma once

namespace amgk {
constexpr int WIN_LMAX = 7;      // longest offset run one staged x window covers
constexpr int WIN_ROWS = 64 + WIN_LMAX - 1;   // rows of one staged x window
// rows of one window a workgroup of four waves copies for all of them; a wave
// takes part in a window when its run's WIN_ROWS-row range starts at most
// WIN_WG_ROWS - WIN_ROWS rows (at most 127) past the window's first row
constexpr int WIN_WG_ROWS = 74;
}  // namespace amgk
