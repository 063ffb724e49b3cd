"""MI355X-native GNN re-ranking hot path (Zhang et al., Section 3.3).

The compute path lives in the HIP library ``librerank.so`` built from
``csrc/``; :mod:`paper_2012_07620_amd.binding` marshals arguments to its
C entry points. Importing this package does not load the library; the first
call does, and raises if the library is missing.
"""
__all__ = ["binding", "synth"]
