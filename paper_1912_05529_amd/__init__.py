"""MI355X-native explicit f-x poststack depth migration.

The compute path is the HIP library ``libmig.so`` (C ABI declared in
``include/mig.h``); :mod:`.mig` marshals torch tensors to it.  :mod:`.synth`
generates seeded synthetic inputs.  Importing this package loads nothing:
the library is opened on first use and its absence is an error.
"""
__all__ = ["mig", "synth"]
