"""MI355X-native overlap-fermion hot path of the lattice Wess-Zumino model.

Sub-modules (imported lazily so that the seeded-input module can be used
without torch or the HIP library):
  inputs    -- seeded synthetic inputs (no arithmetic of the method)
  _lib      -- ctypes binding of libov.so (C ABI of include/ov.h)
  lattice   -- Lattice: sign / apply / solve / force on torch CUDA tensors
  autograd  -- OvForce, the HMC force as a torch.autograd.Function
"""


def __getattr__(name):
    if name in ("Lattice", "solve_batch"):
        from . import lattice
        return getattr(lattice, name)
    if name == "OvForce":
        from .autograd import OvForce
        return OvForce
    raise AttributeError(name)
