"""Sampled sub-block hashing (arXiv 2308.02856) on AMD Instinct MI355X.

The compute path is the HIP library ``libssbh.so`` (C ABI in include/ssbh.h);
``paper_2308_02856_amd.ssbh`` is its thin Python binding.
"""

from . import ssbh  # noqa: F401
