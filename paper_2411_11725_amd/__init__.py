"""MI355X-native nodal finite-difference micromagnetics (HIP / CDNA4).

The compute path lives in the shared library ``libnm.so`` built from
``csrc/``; ``binding`` exposes its C entry points to Python under the same
names.  Importing this package loads nothing: the library is opened on the
first call and a missing build raises immediately.
"""
