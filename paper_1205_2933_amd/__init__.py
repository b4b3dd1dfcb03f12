"""MI355X library for adaptive multigrid on the Shamir domain-wall operator.

The computation lives in ``libmgdwf.so`` (HIP, gfx950) behind the C ABI of
``include/mgdwf.h``; this package is its thin Python binding.  Importing the
package fails loudly if the library has not been built.
"""

from ._lib import *  # noqa: F401,F403
from ._lib import Handle, Handle2D, MgdwfError, make_mg_params, exported_symbols  # noqa: F401
