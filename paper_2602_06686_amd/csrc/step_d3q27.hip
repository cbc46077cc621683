// Fused-step kernels of the D3Q27 lattice (one translation unit per lattice).
#include "step_launch.hpp"

namespace ptrt {

void launch_step_d3q27(const StepLaunch &a) { launch_step_lattice<D3Q27>(a); }

bool launch_step2_d3q27(const StepLaunch &a, double *pass_bytes)
{
    return launch_step2_lattice<D3Q27>(a, pass_bytes);
}

} // namespace ptrt
