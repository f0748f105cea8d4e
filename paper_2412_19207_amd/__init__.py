"""MI355X-native RaNN overlapping-Schwarz least-squares solver.

The compute path lives in the HIP library ``librann_dd.so`` (built from
``csrc/``); ``binding`` exposes its C entry points to Python.  Importing the
package does not load the library; ``binding.load()`` does, and raises if it is
missing.
"""
__all__ = ["binding", "workloads"]
