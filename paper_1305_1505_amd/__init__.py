"""PINOCCHIO collapse-time path on MI355X (gfx950): Python binding of the ``libpin`` C ABI.

The compute path is the HIP library built from ``csrc/``; ``binding`` loads it (and raises if it
is missing) and exposes its entry points under the same names.  ``workloads`` names the
synthetic benchmark workloads.
"""

__all__ = ["binding", "workloads"]
