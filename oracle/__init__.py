"""FP64 CPU oracle of the bilateral filter and of its N-term expanded form.

TEST INFRASTRUCTURE ONLY: imported by tests/, by the smoke check and by the
benchmark's CPU-baseline leg, never by the GPU library.  See fit.py (kernel
expansions) and bfref.c (the filters T1, T2, T3).
"""
from .fit import (spatial_fit, spatial_rectangles, range_fit, range_kernel_approx,
                  haar_family, haar_coefficient, gaussian_integral, truncation_radius,
                  first_m_containing, cosine_coefficients, select_largest, PHI,
                  spatial_fit_2d, spatial_kernel_2d, range_kernel, cell_integrals, KINDS,
                  spatial_fit_table, tabulated_cell_integrals, range_fit_table,
                  piecewise_linear_cosine_coefficients)
from .filters import (Plan, make_plan, make_table_plan, true_bf, true_bf_tab, expanded_brute, expanded_box,
                      correlate_rects, to_unit, expanded_rangebox, expanded_sat3d, box_levels)

__all__ = ["spatial_fit", "spatial_rectangles", "range_fit", "range_kernel_approx",
           "haar_family", "haar_coefficient", "gaussian_integral", "truncation_radius",
           "first_m_containing", "cosine_coefficients", "select_largest", "PHI",
           "spatial_fit_2d", "spatial_kernel_2d", "range_kernel", "cell_integrals", "KINDS",
           "spatial_fit_table", "tabulated_cell_integrals", "range_fit_table",
           "piecewise_linear_cosine_coefficients",
           "Plan", "make_plan", "make_table_plan", "true_bf", "true_bf_tab", "expanded_brute", "expanded_box",
           "correlate_rects", "to_unit", "expanded_rangebox", "expanded_sat3d", "box_levels"]
