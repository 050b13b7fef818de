"""MI355X-native matrix-free NGF + curvature deformable registration.

Submodules (imported on first use, so importing the package loads nothing):

* ``ngf``   - Python binding of the HIP library's C ABI (include/ngfreg.h);
* ``synth`` - seeded synthetic phantoms and displacement fields;
* ``build`` - compiles the gfx950 library in place;
* ``autograd`` - the objective as a torch.autograd.Function.
"""

import importlib

__all__ = ["ngf", "synth", "build", "autograd"]


def __getattr__(name):
    if name in __all__:
        return importlib.import_module(f".{name}", __name__)
    raise AttributeError(name)
