"""libpwadvect: MI355X-native Piacsek-Williams momentum advection.

The compute path is the HIP library ``libpwadvect.so`` (built from ``csrc/``)
behind the C ABI declared in ``include/pwadvect.h``.  This package only
marshals arguments to it:

* ``paper_2010_01545_amd.pwadvect``  -- ctypes binding with the ABI's names
  (``fwd``, ``adj``, ``fwd_adj``, ``pad_periodic``, ``halo_periodic``,
  ``fill_uniform``) on torch device tensors;
* ``paper_2010_01545_amd.autograd``  -- ``PWAdvect``, a torch.autograd.Function
  whose backward is the library's gather-form adjoint;
* ``paper_2010_01545_amd.inputs``    -- seeded synthetic inputs (numpy);
* ``paper_2010_01545_amd.build``     -- hipcc build of the library.

Submodules are imported lazily so that importing the input generators does not
load the GPU library.
"""
import importlib

__all__ = ["pwadvect", "autograd", "inputs", "build"]


def __getattr__(name):
    if name in __all__:
        return importlib.import_module("." + name, __name__)
    raise AttributeError(name)
