"""Workload parameter sets shared by the tests (defined beside the generators)."""
from paper_2405_04229_amd.workload import (ATMO_LAYERED, ATMO_STRAIGHT, RUN_BATCH, RUN_INCLINED,  # noqa: F401
                                           RUN_TELESCOPE, RUN_TINY, SURROGATE_CURVED_HI, SURROGATE_CURVED_LO,
                                           SURROGATE_HI, SURROGATE_LO)
