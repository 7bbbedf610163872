"""MI355X-native interaction-potential + immersed-boundary Lagrangian step.

``native`` binds the C-ABI library ``libipibm.so`` (HIP kernels for gfx950);
``workload`` builds seeded synthetic inputs.  Importing ``native`` fails if the
library is not built: there is no CPU fallback.
"""
