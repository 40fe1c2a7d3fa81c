"""MI355X-native mini-batch kernel k-means (hot path of arXiv 2410.05902)."""
