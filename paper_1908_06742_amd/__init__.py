"""MI355X (gfx950) implementation of the DDF lattice Boltzmann method with local
vorticity extraction (Hajabdollahi & Premnath, arXiv:1908.06742).

The method runs in HIP kernels behind the C ABI of ``libddf.so`` (include/ddf.h and
include/ddf_nn.h); this package is the thin Python binding over it:

- ``Lattice``: one lattice (init, step, extract, reduce, checkpoint);
- ``Batch``: many independent lattices in one persistent, graph-captured launch;
- ``steady``: run-to-steady drivers on the FP64 residual;
- ``surrogate``: the cavity U-Net (BF16 MFMA training and inference) and the warm start;
- ``surrogate_study`` / ``precision_study``: the time-to-steady and 16-bit storage studies.
"""
from ._lib import DDFError, OUTPUTS, STATS, lib  # noqa: F401


def __getattr__(name):
    # torch-dependent classes are imported on first use
    if name == "Lattice":
        from .lattice import Lattice
        return Lattice
    if name == "Batch":
        from .batch import Batch
        return Batch
    raise AttributeError(name)
