"""MI355X (gfx950) deterministic Jet refinement of partitioned hypergraphs (connectivity metric).

The compute path is libjet.so: hand-written HIP kernels behind the C ABI of include/jet.h.  This
package holds its sources (csrc/), its build script and a thin ctypes binding (jet.py).
"""
from .jet import (JET_EHIP, JET_EINVAL, JET_ENOMEM, JET_EOVERFLOW, JET_EUNSUPPORTED, JET_IMBALANCED, JET_OK,
                  JetBatch, JetContext, JetError, TauNet, jet_params_default, jet_tau_features, lib, make_params)

__all__ = ["JetBatch", "JetContext", "JetError", "TauNet", "jet_tau_features", "lib", "make_params", "jet_params_default", "JET_OK", "JET_IMBALANCED",
           "JET_EINVAL", "JET_ENOMEM", "JET_EHIP", "JET_EOVERFLOW", "JET_EUNSUPPORTED"]
