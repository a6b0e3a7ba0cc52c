"""FP64 CPU oracle — TEST INFRASTRUCTURE ONLY.

Only ``tests/``, ``__graft_entry__.smoke()`` and the ``cpu_baseline`` leg of
``bench.py`` may import this package.  The product path (the HIP library and
its Python binding) never imports, links or executes anything in here, and
this package imports nothing from the product path.
"""

from .rsfde_oracle import *  # noqa: F401,F403
from .rsfde_oracle3d import *  # noqa: F401,F403
