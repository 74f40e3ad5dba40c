"""MI355X-native finite-volume solver with learned stencil coefficients."""
