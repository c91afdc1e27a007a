"""MI355X-native Newtonian ray tracing of grating cloaks.

The compute path lives in the HIP library ``libgcloak.so`` (sources under
``csrc/``); ``binding`` marshals torch tensors into its C ABI.  Import
``paper_1012_5107_amd.binding`` for the calls; this package module itself
loads nothing so that the seeded input recipes in ``workloads`` can be used
without a GPU.
"""
__all__ = ["workloads"]
