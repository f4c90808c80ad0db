"""MI355X-native vector-valued Allen-Cahn segmentation (Kay & Tomasi)."""
