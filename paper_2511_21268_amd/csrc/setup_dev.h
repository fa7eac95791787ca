// Device execution of the hierarchy set-up (setup_dev.hip): the same
// hierarchy as build_hierarchy on the host, bit for bit.
#pragma once
#include "host.h"

namespace amgiga {

struct DevSetupInfo {
    int sweeps = 0;         // matching sweeps run
    int rounds_total = 0;   // rounds of locally dominant edges, summed
    int rounds_max = 0;     // and the most in one sweep
};

// Returns 0 or an amg_status code (err set): -1 unsupported input (smoothed
// prolongator, 2^31 or more stored entries, structurally nonsymmetric matrix),
// -3 HIP failure, -4 host allocation failure; otherwise as build_hierarchy.
int build_hierarchy_on_device(const CsrView &K0, const double *w, const SetupParams &prm, HostHierarchy &H,
                              std::string &err, void *stream, DevSetupInfo *info);

}  // namespace amgiga
