"""MI355X (gfx950) implementation of the data-parallel hot path of the
point-neuron cortical simulator of Pastorelli et al. (PDP 2018): LIF+SFA
neurons on a 2-D grid of cortical modules, Gaussian or exponential lateral
connectivity, 1 ms steps with delayed spike fan-out.

The C ABI lives in include/snn.h and libsnn.so (built by build.py); `snn`
is its ctypes binding.  `workloads` holds the seeded network descriptions.
"""
__all__ = ["snn", "workloads", "build"]
