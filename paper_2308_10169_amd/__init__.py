"""libsepso: MI355X-native hot path of SEPSO path planning (grouped tensor-form
PSO with a length + crossing-penalty fitness), its frame loop and batching.

`sepso` is the ctypes binding of the HIP library; `inputs` generates seeded
synthetic workloads.  Importing this package does not touch the GPU.
"""
__all__ = ["sepso", "inputs"]
