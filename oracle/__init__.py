"""FP64 oracle for the interpolation-based 3-D optoacoustic operators.

TEST INFRASTRUCTURE ONLY.  Only tests/, the smoke check in
__graft_entry__.py and the CPU-baseline leg of bench.py may import anything
here.  It shares no code with the HIP library and the HIP library never
calls it.

Parity status of each function against the paper's definitions:
  srt / srt_adj     pinned: uniform-ball and Gaussian closed forms (convergence),
                    brute-force tent-function assembly on tiny grids, adjoint identity
  diff / diff_adj   pinned: polynomial exactness, adjoint identity
  project / backproject  pinned: analytic N-wave convergence, adjoint identity
  fbp               pinned: exact centre value of a centred ball, direct-form equality
"""
