"""MI355X-native semi-global matching (SGM) hot path of the road-disparity pipeline."""
