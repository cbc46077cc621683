// Fused-step kernels of the D2Q9 lattice (one translation unit per lattice).
#include "step_launch.hpp"

namespace ptrt {

void launch_step_d2q9(const StepLaunch &a) { launch_step_lattice<D2Q9>(a); }

bool launch_step2_d2q9(const StepLaunch &a, double *pass_bytes)
{
    return launch_step2_lattice<D2Q9>(a, pass_bytes);
}

} // namespace ptrt
