"""VP-LBM on MI355X: fused D2Q9 BGK + volume penalization step with momentum
exchange and stress integration forces (HIP, gfx950), behind the C ABI of
``include/vplbm.h``.  ``paper_2110_00967_amd.vplbm`` is the ctypes binding."""

__all__ = ["vplbm"]
