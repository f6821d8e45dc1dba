"""MI355X-native concrete race checker for kernels in the minimal OpenCL-style
language of "Detecting Data Races on OpenCL Kernels with Symbolic Execution".

The HIP library (``librc.so``, C ABI in ``include/rc.h``) runs every
work-item of every work-group lockstep over seeded inputs and reports the
non-benign races of every barrier interval; ``binding`` is its Python handle
and ``workloads`` writes the synthetic programs.
"""
