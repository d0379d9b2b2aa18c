"""MI355X-native Swendsen-Wang sweep engine for the Ising model.

The compute path is the HIP library ``libswgpu.so`` (C ABI declared in
``include/sw_api.h``); ``paper_0808_2109_amd.swgpu`` is its thin ctypes
binding.  ``paper_0808_2109_amd.workloads`` holds the seeded input and
workload generators.  Importing this package loads nothing by itself.
"""
__all__ = ["swgpu", "workloads"]
