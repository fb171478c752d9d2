// xf_react.hip -- the reaction step's launcher for one species count
// (compiled once per N with -DXF_NS=N, like xf_ns.hip).
//
// Built with machine-level loop-invariant code motion off: the kernel's
// sub-step loop calls exp, expm1 and log, whose FP64 polynomial constants
// cannot be instruction operands on this target, and hoisting their
// materialisation out of the loop keeps some forty of them live across it,
// which at four waves per SIMD spills them to scratch and reloads them on
// every call; left in the loop they cost a few scalar moves each.
#include "xf_reaction.hpp"

#ifndef XF_NS
#error "compile with -DXF_NS=<species count>"
#endif

namespace xf {

template <>
hipError_t react_launch<XF_NS>(const LaunchCtx &c, double *U, const ReactK *rk, double dt, const double *dt_dev,
                               double scale, int n_sub, hipStream_t s) {
    const long long n = (long long)c.g.nx * c.g.ny * c.g.nz;
    const unsigned blocks = (unsigned)((n + 255) / 256);
    hipLaunchKernelGGL(k_react<XF_NS>, dim3(blocks), dim3(256), 0, s, U, c.g, rk, dt, dt_dev, scale, n_sub,
                       c.status);
    return hipGetLastError();
}

}  // namespace xf
