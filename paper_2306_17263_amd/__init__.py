"""MI355X stepper for the compact fourth-order staggered scheme of Versano,
Turkel and Tsynkov (arXiv 2306.17263).  The scheme runs in the gfx950
library libc4m.so (C ABI in include/c4m.h); this package only marshals
arguments, with PyTorch providing device memory and streams."""
from ._lib import (  # noqa: F401
    C4mError, EXPORTS, load, OK, EINVAL, ENOMEM, EDEVICE, ESTATE, ENOCONV, EUNSTABLE, ENONFINITE,
    FLAG_ALLOW_ANY_CFL, FLAG_CHECK_FINITE, FLAG_PROFILE, FLAG_DIRECT,
)
from .problem import Problem, make_config, workspace_bytes  # noqa: F401
from .batch import Batch  # noqa: F401
