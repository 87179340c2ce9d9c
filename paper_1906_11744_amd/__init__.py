"""MI355X-native batched Kalman-filter track fit, combinatorial finder and fit adjoint.

The compute lives in libkf.so (HIP kernels for gfx950 behind include/kf.h); this
package is its binding.  See kf.Context.
"""
from .autograd import FitChi2, fit_chi2  # noqa: F401
from .kf import Context, KfError  # noqa: F401
