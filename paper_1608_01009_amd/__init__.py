"""MI355X-native explicit electromagnetic PIC step (arXiv:1608.01009).

* ``paper_1608_01009_amd.pic``: binding of the HIP library ``libpic_hip.so``
  (C ABI in ``include/pic.h``).
* ``paper_1608_01009_amd.workloads``: seeded synthetic plasma inputs.
* ``paper_1608_01009_amd.build``: hipcc build of the library for gfx950.

Importing the package loads nothing; the library is opened on first use.
"""

__all__ = ["pic", "workloads", "build"]
